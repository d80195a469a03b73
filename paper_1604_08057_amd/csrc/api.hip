// C ABI of the tslov library (declared in include/tslov.h): context and
// workspace management, and the host drivers of the TSL forward pass, the
// projected-matrix Newton step and the reverse-mode pass for dS/dU.  Every
// driver works on a batch of sources held in workspace slots; a single-source
// call is a batch of one.
#include "tslov.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "ritz.h"

using tslov::Coef;
using tslov::DenseWork;
using tslov::Geom;
using tslov::kMaxBatch;
using tslov::SrcList;
using tslov::Work;
using tslov::Z;
using tslov::ZD;

namespace {

thread_local std::string g_err;

tslov_status fail(tslov_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(x)                                                                               \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) return fail(TSLOV_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CHK(x)                               \
    do {                                     \
        tslov_status s_ = (x);               \
        if (s_ != TSLOV_OK) return s_;       \
    } while (0)

struct Buf {
    void* p = nullptr;
    size_t n = 0;
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

tslov_status ensure(Buf& b, size_t bytes) {
    if (b.n >= bytes && b.p) return TSLOV_OK;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(TSLOV_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    b.n = bytes;
    return TSLOV_OK;
}

void release(Buf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kMaxK = 1024;
constexpr int kMaxDeflSet = 256;
constexpr int kTimingClasses = 3;
constexpr int kMaxSources = 1 << 20;

// Site-block order of the colour-split and force kernels (Geom::sbmap; workgroup i
// runs on XCD i % 8).  When one XCD's share of a t-slice, at the stencil pair's
// bytes per site, fits in half an XCD's L2, each XCD takes the same segment of
// every t-slice with t outermost: a site's t-neighbours were then touched one
// segment earlier on the same L2, and only z-neighbours across segment edges come
// from memory.  Otherwise each XCD takes a contiguous run of the lattice.  The lists
// are padded to equal length with -1 (idle workgroups).
std::vector<int> site_block_order(const Geom& g, int& nwg) {
    const int nsb = tslov::nsb_pad(g.V), kx = tslov::kXcd;
    const long long V3 = (long long)g.nx * g.ny * g.nz;
    constexpr double kPairBytesPerSite = 1728.0;          // links + six fields, FP64
    constexpr double kL2Budget = 2.0 * 1024.0 * 1024.0;   // half of an XCD's 4 MB
    const bool seg = (double)V3 / kx * kPairBytesPerSite <= kL2Budget;
    std::vector<std::vector<int>> per(kx);
    for (int b = 0; b < nsb; ++b) {
        const long long pos = ((long long)b * tslov::kSites) % V3;   // first site's place in its slice
        per[seg ? (int)(pos * kx / V3) : b / (nsb / kx)].push_back(b);
    }
    size_t m = 0;
    for (const auto& v : per) m = std::max(m, v.size());
    nwg = (int)m * kx;
    std::vector<int> map((size_t)nwg, -1);
    for (int x = 0; x < kx; ++x)
        for (size_t i = 0; i < per[x].size(); ++i) map[i * kx + x] = per[x][i];
    return map;
}

}  // namespace

// Device memory of the allocation-free operator entry point: the two structure-
// of-arrays staging fields (input and output of the stencil) for lattices of up
// to kScratchBytes / (2 * 12 * sizeof(complex)) sites.  Each device holds its own
// copy while the process lives; host code reaches it only through the address
// hipGetSymbolAddress returns for that device (the array's name is a host-side
// stand-in, not a device address).
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device `dev`, looked up once per device.
tslov_status scratch_address(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(TSLOV_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(TSLOV_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return TSLOV_OK;
}
}  // namespace

// A captured launch sequence and the key (list, sizes, buffers, launch shapes) it
// was captured for.
struct LoopGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<char> key;
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        key.clear();
    }
};

struct tslov_ctx {
    Geom g{};
    double kappa = 0.0, mu = 0.0;
    int antiperiodic = 1, precision = TSLOV_FP64;
    hipStream_t st = nullptr;
    int device = 0;
    char* scratch = nullptr;   // this device's scratch array (allocation-free operator)
    size_t lds_max = 65536;
    int links_set = 0;
    int diag = 0;    // tslov_set_diagnostics flags
    int nest_m = 0;  // inner Krylov size of the nested projected-matrix step (0: plain)
    Buf blk;         // block-matrix process: 14 working fields, 2k basis fields, partials
    Buf bdefl;       // deflated block process: dH R_i, dR_i, the shifted solutions, temporaries, coefficients
    Buf deflb;       // batched deflated derivative: projected sources, TSL source gradients and outputs
    Buf curdefl;     // deflated current estimator: g5 xi, per-source dU, y, dpsi and U(1) projections
    Buf nestbuf;     // its inner basis, vectors and coefficients
    Buf U64, U32;
    Buf badflag;     // device int: a non-finite link element was seen
    Buf sbmap;       // Geom::sbmap
    Buf opf;         // two working-precision fields for the plain operator
    // batch workspace: per slot, kcap steps of v, w, a = Hv, b = H^dag w (and
    // abar, sbar for the derivative), kNF fields and kNP partial arrays
    Buf basisV, basisW, basisA, basisB, abarS, sbarS;
    Buf fields, part, coefmem;
    Buf dense, denseInt, densePart, denseDelta;
    Buf gpart, gsrc;
    Buf bout;        // per-entry canonical y and dpsi (Ward check)
    Buf wardp;       // Ward block maxima
    Buf canon;       // canonical spinors: projected source, partial result, error estimate
    Buf trial;       // the tuning run's trial vector (1, ..., 1)
    Buf solvebuf;    // overlap solve: r, z, p, w and a g5 copy (canonical)
    Buf physbuf;     // physical current: chi_s and the probes g5 chi_s, i g5 chi_s
    Buf deflw;       // deflation coefficients, signs and partial sums
    Buf deflx;       // deflated derivative: R^H eta, R^H psibar, q, -q and dot partials
    Buf cgf, cgp, cgs;   // shifted solves: fields, partial sums, per-system scalars
    double* host_part = nullptr;  // pinned
    int host_part_n = 0;
    int slots = 0, kcap = 0, grad_cap = 0;   // shape of the batch workspace
    // recompute mode: steps of v, w, a, b, abar, sbar held per slot (a ring; 0:
    // all kcap steps), the segment length and the checkpoint fields
    int ring = 0, ring_m = 0;
    Buf ckpt;
    // captured forward and reverse loops (tslov_set_graphs)
    int graphs = 0;
    LoopGraph gfwd, gbwd;
    int dslots = 0, dkcap = 0;               // shape of the dense workspace
    Coef coef{};
    int timing = 0;            // 0 off, N: time every N-th launch of each class
    long long tcount[kTimingClasses] = {0, 0, 0};
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[kTimingClasses];
    // entries per workgroup of the colour-split pair kernels ([0] forward, [1]
    // reverse): the timed pick (0 = none yet) and the list length it was timed
    // at; pair_ns_forced > 0 overrides the pick
    int pair_ns[2] = {0, 0};
    int pair_ns_n[2] = {0, 0};
    int pair_ns_forced = 0;
    // t-slices per chunk of the t-march operator: the timed pick (0: none yet,
    // -1: the operator does not march on this lattice) and a forced value
    int tm_T = 0, tm_T_forced = 0;
    // operator form of the shifted solves of the deflated derivative (tslov::kCgOp*)
    int cg_op = tslov::kCgOpTmarch;

    int nblk() const { return tslov::grid_for(g.V); }
    size_t field_elems() const { return (size_t)12 * g.ldv; }
    size_t zsize() const { return precision == TSLOV_MIXED ? sizeof(Z<float>) : sizeof(ZD); }
    // bytes of one complex link element as the stencils read it
    size_t lsize() const { return precision == TSLOV_FP64 ? sizeof(ZD) : sizeof(Z<float>); }
    size_t field_bytes() const { return field_elems() * zsize(); }
    int pstride() const { return 8 * tslov::np_max(g.V); }
};

namespace {

// ---------------------------------------------------------------- timing
// Event pair for one launch of a timing class, recorded by the launch's own
// dispatch (hipExtLaunchKernel), or none when timing is off or the launch is not
// in the sample.
struct TimedLaunch {
    tslov::Timing t;
    TimedLaunch(tslov_ctx* c, int cls) {
        if (!c->timing) return;
        // every c->timing-th launch of the class
        if (c->tcount[cls]++ % c->timing != 0) return;
        hipEvent_t a = take(c), b = take(c);
        if (!a || !b) return;
        t.a = a;
        t.b = b;
        c->ev_used[cls].push_back({a, b});
    }
    static hipEvent_t take(tslov_ctx* c) {
        if (c->ev_free.empty()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            return e;
        }
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
};

// ---------------------------------------------------------------- launch-shape tuner
// Entries per workgroup of a colour-split pair kernel (1, 2 or 4).  The choice
// only decides how many entries share each link load; every entry's arithmetic
// and partial-sum slots are the same for all of them, so it changes the time of
// a step, never its result.  The first steps over a list of the target length
// cycle through the candidates (at most the list length) with an event pair
// around each launch, kTuneReps rounds; the fastest of each candidate's best
// times becomes the pick, kept for the context's later calls.  A pick timed on a
// list shorter than 4 is timed again once a list of 4 or more comes along.
struct PairTuner {
    static constexpr int kCand[3] = {1, 2, 4};
    static constexpr int kTuneReps = 3;
    tslov_ctx* c;
    int cls, target, ncand = 0, step = 0;
    std::vector<hipEvent_t> ev;

    PairTuner(tslov_ctx* ctx, int which, int n_target) : c(ctx), cls(which), target(n_target) {
        if (c->pair_ns_forced || tslov::colour_grid(c->g.V) || target < 2) return;
        if (c->pair_ns[cls] && !(c->pair_ns_n[cls] < 4 && target >= 4)) return;
        ncand = target >= 4 ? 3 : 2;
        ev.assign((size_t)2 * ncand * kTuneReps, nullptr);
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                e = nullptr;
                ncand = 0;
            }
        if (!ncand) release();
    }
    ~PairTuner() { release(); }
    void release() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        ev.clear();
    }
    static int fit(int ns, int n) {
        while (ns > 1 && ns > n) ns /= 2;
        return ns;
    }
    bool tuning(int n) const { return ncand && n == target && step < ncand * kTuneReps; }
    bool active() const { return ncand != 0; }
    // entries per workgroup for the next launch over a list of n entries
    int ns(int n) const {
        if (c->pair_ns_forced) return fit(c->pair_ns_forced, n);
        if (tuning(n)) return kCand[step % ncand];
        return fit(c->pair_ns[cls] ? c->pair_ns[cls] : 1, n);
    }
    void before(int n) {
        if (tuning(n)) (void)hipEventRecord(ev[2 * step], c->st);
    }
    void after(int n) {
        if (!tuning(n)) return;
        (void)hipEventRecord(ev[2 * step + 1], c->st);
        if (++step < ncand * kTuneReps) return;
        float best[3] = {1e30f, 1e30f, 1e30f};
        if (hipEventSynchronize(ev.back()) != hipSuccess) {
            (void)hipGetLastError();
            ncand = 0;
            return;
        }
        for (int i = 0; i < step; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess)
                best[i % ncand] = std::min(best[i % ncand], ms);
        }
        int pick = 0;
        for (int q = 1; q < ncand; ++q)
            if (best[q] < best[pick]) pick = q;
        c->pair_ns[cls] = kCand[pick];
        c->pair_ns_n[cls] = target;
        ncand = 0;
    }
};

// ---------------------------------------------------------------- captured loops
// The forward and reverse Lanczos loops of a source list are kernel launches only,
// and every decision inside them (breakdown, retirement) is taken on the device, so
// with graphs on each loop is captured once as a HIP graph and replayed while the
// list, the sizes, the buffers and the launch shapes stay the same (the key holds
// exactly these).  Not while kernels are timed, while the pair-kernel shape is still
// being timed, in recompute mode (its checkpoints are copies) or on the null stream.
struct LoopKey {
    std::vector<char> b;
    template <typename T>
    LoopKey& add(const T& v) {
        const char* p = reinterpret_cast<const char*>(&v);
        b.insert(b.end(), p, p + sizeof(T));
        return *this;
    }
    LoopKey& list(const SrcList& L) {
        add(L.n);
        for (int e = 0; e < L.n; ++e) add(L.slot[e]).add(L.k[e]);
        return *this;
    }
    // the workspace, links and launch shapes the loops' kernels receive
    template <typename R, typename RL>
    LoopKey& buffers(const tslov_ctx* c, const Work<R>& wk, const Z<RL>* U, int cls) {
        add(wk.V).add(wk.W).add(wk.A).add(wk.B).add(wk.AB).add(wk.SB).add(wk.F).add(wk.part);
        add(wk.fe).add(wk.kcap).add(wk.ring).add(wk.pstride);
        add(c->coefmem.p).add(c->slots).add(c->kcap).add(U).add(c->mu);
        return add(c->pair_ns[cls]).add(c->pair_ns_forced);
    }
};

bool graphs_usable(const tslov_ctx* c) { return c->graphs && !c->timing && c->st && !c->ring; }

template <typename F>
tslov_status run_captured(tslov_ctx* c, LoopGraph& lg, const LoopKey& key, F&& launches) {
    if (!lg.exec || lg.key != key.b) {
        lg.reset();
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
        const tslov_status st = launches();
        const hipError_t e = hipStreamEndCapture(c->st, &graph);
        if (st != TSLOV_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        HIPCHK(e);
        const hipError_t ei = hipGraphInstantiate(&lg.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            lg.exec = nullptr;
            return fail(TSLOV_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        }
        lg.key = key.b;
    }
    HIPCHK(hipGraphLaunch(lg.exec, c->st));
    return TSLOV_OK;
}

tslov_status ensure_host_part(tslov_ctx* c, int n) {
    if (c->host_part_n >= n) return TSLOV_OK;
    if (c->host_part) (void)hipHostFree(c->host_part);
    c->host_part = nullptr;
    c->host_part_n = 0;
    HIPCHK(hipHostMalloc((void**)&c->host_part, (size_t)n * sizeof(double), hipHostMallocDefault));
    c->host_part_n = n;
    return TSLOV_OK;
}

// ---------------------------------------------------------------- batch workspace
size_t coef_bytes(int slots, int kcap) {
    const size_t n = (size_t)kcap + 2;
    return (size_t)slots * (n * (7 * sizeof(ZD) + 4 * sizeof(double)) + 16 * sizeof(int) + 16 * sizeof(double));
}

void carve_coef(tslov_ctx* c, int slots, int kcap) {
    const size_t n = (size_t)kcap + 2, S = (size_t)slots;
    char* p = c->coefmem.as<char>();
    auto take = [&](size_t b) {
        char* q = p;
        p += b;
        return q;
    };
    Coef& cf = c->coef;
    cf.alpha = (ZD*)take(S * n * sizeof(ZD));
    cf.gamma = (ZD*)take(S * n * sizeof(ZD));
    cf.h = (ZD*)take(S * n * sizeof(ZD));
    cf.c = (ZD*)take(S * n * sizeof(ZD));
    cf.abar_T = (ZD*)take(S * n * sizeof(ZD));
    cf.gbar_T = (ZD*)take(S * n * sizeof(ZD));
    cf.gbar_tot = (ZD*)take(S * n * sizeof(ZD));
    cf.beta = (double*)take(S * n * sizeof(double));
    cf.anorm2 = (double*)take(S * n * sizeof(double));
    cf.bbar_T = (double*)take(S * n * sizeof(double));
    cf.bbar_tot = (double*)take(S * n * sizeof(double));
    cf.misc = (double*)take(S * 16 * sizeof(double));
    cf.status = (int*)take(S * 16 * sizeof(int));
    cf.n = (int)n;
}

// Steps of basis vectors held per slot for segments of m steps (m = 0: all kcap):
// a segment's reverse steps read v, w at j0 - 1 .. j1 + 1.
int ring_steps(int kcap, int m) { return (m > 0 && m + 2 < kcap) ? m + 2 : 0; }
int n_segments(int kcap, int m) { return (kcap + m - 1) / m; }

// Workspace for `slots` sources of up to kcap steps (grad: with the reverse-pass
// arrays; m > 0: recompute mode with segments of m steps).
tslov_status ensure_work(tslov_ctx* c, int slots, int kcap, int grad, int m = 0) {
    const int ring = ring_steps(kcap, m);
    if (c->slots == slots && c->kcap == kcap && c->grad_cap >= grad && c->ring == ring &&
        (!ring || c->ring_m == m) && c->coefmem.p)
        return TSLOV_OK;
    c->slots = 0;   // invalid until every buffer has the new shape
    const size_t fb = c->field_bytes();
    const size_t per = (size_t)slots * (ring ? ring : kcap) * fb;
    if (ring) CHK(ensure(c->ckpt, (size_t)slots * n_segments(kcap, m) * 4 * fb));
    c->ring = ring;
    c->ring_m = ring ? m : 0;
    CHK(ensure(c->basisV, per));
    CHK(ensure(c->basisW, per));
    CHK(ensure(c->basisA, per));
    CHK(ensure(c->basisB, per));
    if (grad) {
        CHK(ensure(c->abarS, per));
        CHK(ensure(c->sbarS, per));
    }
    CHK(ensure(c->fields, (size_t)slots * tslov::kNF * fb));
    CHK(ensure(c->part, (size_t)slots * tslov::kNP * c->pstride() * sizeof(double)));
    CHK(ensure(c->coefmem, coef_bytes(slots, kcap)));
    carve_coef(c, slots, kcap);
    c->slots = slots;
    c->kcap = kcap;
    c->grad_cap = grad;
    return TSLOV_OK;
}

template <typename R>
Work<R> work(const tslov_ctx* c) {
    Work<R> w;
    w.V = c->basisV.as<Z<R>>();
    w.W = c->basisW.as<Z<R>>();
    w.A = c->basisA.as<Z<R>>();
    w.B = c->basisB.as<Z<R>>();
    w.AB = c->abarS.as<Z<R>>();
    w.SB = c->sbarS.as<Z<R>>();
    w.F = c->fields.as<Z<R>>();
    w.part = c->part.as<double>();
    w.fe = c->field_elems();
    w.kcap = c->ring ? c->ring : c->kcap;
    w.pstride = c->pstride();
    w.ring = c->ring ? 1 : 0;
    return w;
}

// The link copy the stencils read: float64, or float32 for TSLOV_MIXED (float
// fields) and TSLOV_FP32_LINKS (float64 fields).
template <typename RL>
const Z<RL>* links(const tslov_ctx* c) {
    if constexpr (sizeof(RL) == sizeof(double)) return c->U64.as<Z<RL>>();
    else return c->U32.as<Z<RL>>();
}

// Device bytes one source of up to kcap steps needs (workspace sizing).
// Chunks of steps the force contraction splits each entry into (its partials are
// summed afterwards): about 2^18 threads in all, and at least 16 chunks so that a
// large lattice does not leave each thread a loop over every step.  A function of
// the lattice only, so an entry's result does not depend on its batch.
int force_chunks(int V) { return std::max(16, std::min((1 << 18) / (4 * V), 64)); }

size_t bytes_per_source(const tslov_ctx* c, int kcap, int grad, int m = 0) {
    const size_t fb = c->field_bytes();
    const int ring = ring_steps(kcap, m);
    size_t b = (size_t)(grad ? 6 : 4) * (ring ? ring : kcap) * fb + (size_t)tslov::kNF * fb;
    if (ring) b += (size_t)4 * n_segments(kcap, m) * fb;
    b += (size_t)tslov::kNP * c->pstride() * sizeof(double) + coef_bytes(1, kcap);
    b += (size_t)6 * kcap * kcap * sizeof(ZD) + (size_t)tslov::dense_pstride(kcap) * sizeof(double);
    if (grad)
        b += (size_t)(force_chunks(c->g.V) + 1) * 36 * c->g.ldv * sizeof(ZD) + (size_t)2 * 12 * c->g.V * sizeof(ZD);
    return b;
}

size_t held_bytes(const tslov_ctx* c) {
    size_t t = 0;
    for (const Buf* b : {&c->basisV, &c->basisW, &c->basisA, &c->basisB, &c->abarS, &c->sbarS, &c->fields, &c->part,
                         &c->dense, &c->gpart, &c->bout, &c->ckpt})
        t += b->n;
    return t;
}

// Sources per batch: as many as fit in ~80% of the device memory not otherwise in use.
int batch_capacity(const tslov_ctx* c, int kcap, int grad, int m = 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    const double avail = 0.8 * (double)(fr + held_bytes(c));
    const double per = (double)bytes_per_source(c, kcap, grad, m);
    const int n = (int)std::floor(avail / per);
    return std::max(1, std::min(n, kMaxBatch));
}

// Sources per group: the capacity estimate, except that a workspace already
// holding within a quarter of that many sources at this size is reused as it is.
// The estimate follows the free memory, which moves between calls, and growing
// the workspace means reallocating many GB inside the call.
int group_size(const tslov_ctx* c, int kcap, int grad, int m, int remaining) {
    int cap = batch_capacity(c, kcap, grad, m);
    const int ring = ring_steps(kcap, m);
    const size_t per_slot = (size_t)(ring ? ring : kcap) * c->field_bytes();
    const int held = c->basisV.p && per_slot ? (int)std::min<size_t>(c->basisV.n / per_slot, kMaxBatch) : 0;
    if (held >= 1 && cap > held && 4 * (cap - held) <= held) cap = held;
    return std::min(cap, remaining);
}

// ---------------------------------------------------------------- source lists
// Entries in slots 0..n-1 sorted by decreasing k.
SrcList make_list(const std::vector<int>& src, const std::vector<int>& k) {
    SrcList L{};
    L.n = (int)src.size();
    for (int e = 0; e < L.n; ++e) {
        L.slot[e] = e;
        L.src[e] = src[e];
        L.k[e] = k[e];
        L.flag[e] = 0;
    }
    return L;
}

SrcList prefix(const SrcList& L, int n) {
    SrcList o = L;
    o.n = n;
    return o;
}

SrcList range(const SrcList& L, int b, int e) {
    SrcList o{};
    o.n = e - b;
    for (int i = b; i < e; ++i) {
        o.slot[i - b] = L.slot[i];
        o.src[i - b] = L.src[i];
        o.k[i - b] = L.k[i];
        o.flag[i - b] = L.flag[i];
    }
    return o;
}

// ---------------------------------------------------------------- forward
struct EntryStatus {
    int k_used = 0, breakdown = 0, step = 0;
    double norm_x = 0.0, S = 0.0;
    int iters = 0, flags = 0, cg_iters = 0;
    double biorth = 0.0, eps_A = NAN;
    tslov::RitzSummary ritz{NAN, NAN, 0};
};

// Eigenvalues of every entry's T_k on host threads, overlapping the device work
// that follows the forward pass (the dense step and the reverse pass).  The
// coefficient arrays are host copies laid out as on the device ([slot][n], step j
// at index j).
struct RitzJobs {
    std::vector<ZD> alpha, gamma;
    std::vector<double> beta;
    int n = 0;
    std::vector<int> kk, slot;
    std::vector<tslov::RitzSummary> out;
    std::vector<std::thread> th;
    std::atomic<int> next{0};
    void start(const std::vector<int>& k_used, const std::vector<int>& slots) {
        kk = k_used;
        slot = slots;
        out.assign(kk.size(), tslov::RitzSummary{NAN, NAN, 0});
        next = 0;
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const int nt = (int)std::min<size_t>(kk.size(), std::min(hw, 16u));
        // one entry: its divide-and-conquer halves run on threads of their own
        const int inner = kk.size() == 1 ? 4 : 1;
        for (int t = 0; t < nt; ++t)
            th.emplace_back([this, inner] {
                for (int e; (e = next++) < (int)kk.size();) {
                    if (kk[e] < 1) continue;
                    const size_t o = (size_t)slot[e] * n + 1;   // step 1 of the slot
                    out[e] = tslov::ritz_summary(kk[e], reinterpret_cast<const double*>(&alpha[o]), &beta[o],
                                                 reinterpret_cast<const double*>(&gamma[o]), inner);
                }
            });
    }
    void join() {
        for (auto& t : th) t.join();
        th.clear();
    }
    ~RitzJobs() { join(); }
};

// A Ritz value on the imaginary axis (relative to the size of T_k) leaves the sign
// of the projected matrix undefined (Sec. 2, after eq. spectral_form).
constexpr double kSignAxisTol = 1e-12;
tslov_status check_ritz(const EntryStatus& s) {
    if (s.k_used > 0 && s.ritz.min_abs_re <= kSignAxisTol * s.ritz.norm_T)
        return fail(TSLOV_ERR_SIGN_UNDEFINED, "a Ritz value of the projected matrix lies on Re z = 0 (|Re theta| = " +
                                                  std::to_string(s.ritz.min_abs_re) + ")");
    return TSLOV_OK;
}

// Recompute mode: the state before forward step j0 = 1 + seg m of every entry of
// L (the residuals r, s of step j0 - 1 and v_{j0-1}, w_{j0-1}), saved (restore = 0)
// to or restored (restore = 1) from checkpoint seg of the entry's slot.
template <typename R>
tslov_status checkpoint(tslov_ctx* c, const SrcList& L, int seg, int j0, int restore) {
    const Work<R> wk = work<R>(c);
    const size_t fb = c->field_bytes();
    const int nseg = n_segments(c->kcap, c->ring_m);
    for (int e = 0; e < L.n; ++e) {
        const int slot = L.slot[e];
        char* base = c->ckpt.as<char>() + ((size_t)slot * nseg + seg) * 4 * fb;
        void* live[4] = {wk.f(slot, 2), wk.f(slot, 3), wk.v(slot, j0 - 1), wk.w(slot, j0 - 1)};
        for (int i = 0; i < 4; ++i) {
            void* saved = base + (size_t)i * fb;
            HIPCHK(hipMemcpyAsync(restore ? live[i] : saved, restore ? saved : live[i], fb, hipMemcpyDeviceToDevice,
                                  c->st));
        }
    }
    return TSLOV_OK;
}

// Lanczos process for every entry of L (slots 0..n-1, k in decreasing order);
// psi and eta canonical arrays indexed by src (eta nullable; eta_g5: eta = g5 psi).
template <typename R, typename RL>
tslov_status forward(tslov_ctx* c, const SrcList& L, const ZD* psi, const ZD* eta, int eta_g5,
                     std::vector<EntryStatus>& es, RitzJobs* jobs = nullptr) {
    const Geom& g = c->g;
    const Work<R> wk = work<R>(c);
    std::vector<int> init((size_t)16 * L.n, 0);
    for (int e = 0; e < L.n; ++e) init[(size_t)16 * L.slot[e] + 1] = L.k[e];
    HIPCHK(hipMemcpyAsync(c->coef.status, init.data(), init.size() * sizeof(int), hipMemcpyHostToDevice, c->st));
    tslov::launch_sources_to_soa<R>(psi, 0, 0, wk, L, g, c->st);
    if (eta) tslov::launch_sources_to_soa<R>(eta, 1, eta_g5, wk, L, g, c->st);
    const Z<RL>* U = links<RL>(c);
    const int kmax = L.k[0];
    PairTuner tune(c, 0, L.n);
    const int m = c->ring ? c->ring_m : 0;
    auto loop = [&]() -> tslov_status {
        int n = L.n;
        for (int j = 1; j <= kmax; ++j) {
            while (n > 0 && L.k[n - 1] < j) --n;
            const SrcList Lj = prefix(L, n);
            if (m && j > 1 && (j - 1) % m == 0) CHK(checkpoint<R>(c, Lj, (j - 1) / m, j, 0));
            tune.before(n);
            tslov::launch_fwd_pair<R, RL>(U, g, c->kappa, c->mu, wk, Lj, c->coef, j, eta ? 1 : 0, tune.ns(n), c->st,
                                      TimedLaunch(c, 0).t);
            tune.after(n);
            tslov::launch_recur<R>(g, wk, Lj, c->coef, j, c->st);
        }
        return TSLOV_OK;
    };
    if (graphs_usable(c) && !tune.active()) {
        LoopKey key;
        key.list(L).add(kmax).add(eta ? 1 : 0).buffers(c, wk, U, 0);
        CHK(run_captured(c, c->gfwd, key, loop));
    } else {
        CHK(loop());
    }
    const int nbb = tslov::launch_biorth<R>(g, wk, L, c->coef, c->st);
    HIPCHK(hipGetLastError());
    // slots 0..nslot-1 hold the list's entries
    int nslot = 0;
    for (int e = 0; e < L.n; ++e) nslot = std::max(nslot, L.slot[e] + 1);
    CHK(ensure_host_part(c, 4 * nbb * L.n));
    std::vector<int> st((size_t)16 * nslot);
    std::vector<double> misc((size_t)16 * nslot);
    HIPCHK(hipMemcpyAsync(st.data(), c->coef.status, st.size() * sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(misc.data(), c->coef.misc, misc.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
    for (int e = 0; e < L.n; ++e)
        HIPCHK(hipMemcpyAsync(c->host_part + (size_t)4 * nbb * e, wk.p(L.slot[e], 3), (size_t)4 * nbb * sizeof(double),
                              hipMemcpyDeviceToHost, c->st));
    if (jobs) {
        const size_t n = (size_t)c->coef.n * nslot;
        jobs->n = c->coef.n;
        jobs->alpha.resize(n);
        jobs->gamma.resize(n);
        jobs->beta.resize(n);
        HIPCHK(hipMemcpyAsync(jobs->alpha.data(), c->coef.alpha, n * sizeof(ZD), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(jobs->gamma.data(), c->coef.gamma, n * sizeof(ZD), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(jobs->beta.data(), c->coef.beta, n * sizeof(double), hipMemcpyDeviceToHost, c->st));
    }
    HIPCHK(hipStreamSynchronize(c->st));
    es.assign(L.n, EntryStatus());
    for (int e = 0; e < L.n; ++e) {
        const int* s = &st[(size_t)16 * L.slot[e]];
        if (s[2] == 3) return fail(TSLOV_ERR_ARG, "a source is not finite");
        es[e].k_used = s[1];
        es[e].breakdown = s[2];
        es[e].step = s[3];
        es[e].norm_x = misc[(size_t)16 * L.slot[e]];
        // |w_1^H v_k| + |w_k^H v_1| with v_1 = w_1 = x/|x|, from the fixed-order block sums
        double d[4] = {0.0, 0.0, 0.0, 0.0};
        const double* pp = c->host_part + (size_t)4 * nbb * e;
        for (int b = 0; b < nbb; ++b)
            for (int i = 0; i < 4; ++i) d[i] += pp[4 * b + i];
        es[e].biorth = es[e].norm_x > 0.0 ? (std::hypot(d[0], d[1]) + std::hypot(d[2], d[3])) / es[e].norm_x : 0.0;
    }
    if (jobs) {
        std::vector<int> ku(L.n), sl(L.n);
        for (int e = 0; e < L.n; ++e) {
            ku[e] = es[e].breakdown == 2 ? 0 : es[e].k_used;
            sl[e] = L.slot[e];
        }
        jobs->start(ku, sl);
    }
    return TSLOV_OK;
}

// ---------------------------------------------------------------- projected-matrix step
tslov_status ensure_dense(tslov_ctx* c, int slots, int kcap, DenseWork& w) {
    const size_t kk = (size_t)kcap * kcap;
    const int ps = tslov::dense_pstride(kcap);
    CHK(ensure(c->dense, (size_t)slots * 8 * kk * sizeof(ZD)));
    CHK(ensure(c->denseInt, (size_t)slots * 2 * kcap * sizeof(int)));
    CHK(ensure(c->densePart, (size_t)slots * ps * sizeof(double)));
    CHK(ensure(c->denseDelta, (size_t)slots * 4 * sizeof(double)));
    CHK(ensure_host_part(c, 4 * slots + 8));
    ZD* d = c->dense.as<ZD>();
    const size_t S = (size_t)slots;
    w.X = d;
    w.Y = d + S * kk;
    w.Wk = d + 2 * S * kk;
    w.Xinv = d + 3 * S * kk;
    w.Zt = d + 4 * S * kk;
    w.Y2 = d + 5 * S * kk;
    w.P2 = d + 6 * S * kk;
    w.Y3 = d + 7 * S * kk;
    w.rowperm = c->denseInt.as<int>();
    w.part = c->densePart.as<double>();
    w.delta = c->denseDelta.as<double>();
    w.kk = kk;
    w.kcap = kcap;
    w.npart_max = tslov::grid_for((int)kk, 256);
    w.pstride = ps;
    c->dslots = slots;
    c->dkcap = kcap;
    return TSLOV_OK;
}

int choose_nb(const tslov_ctx* c, int k) {
    for (int nb : {16, 8, 4, 2, 1})
        if ((size_t)(k * (nb + 1)) * sizeof(ZD) + (size_t)k * sizeof(int) + 2048 <= c->lds_max) return nb;
    return 1;
}

// Newton iteration on X (and Y) of every entry of L (k = size, decreasing) until
// each entry's relative step falls to rounding level.  Scaled inverse-based steps
// first; the inverse-free step takes over once |I - X^2|_F < kNsSafe, where it is
// guaranteed to converge quadratically (checked after inverse-based steps whose
// predecessor moved X by less than kResidCheck), or once the step is below
// kNsSwitch; it hands back if it ever fails to contract.  iters[e] receives the
// step count.
constexpr double kNsSwitch = 1e-2;
constexpr double kNsSafe = 0.9;
constexpr double kResidCheck = 2.0;

tslov_status newton(tslov_ctx* c, const SrcList& L, int grad, const DenseWork& w, std::vector<int>& iters,
                    int tridiag_start, std::vector<int>* stagnated = nullptr) {
    struct St {
        int scaling = 1, extra = 0, done = 0, it = 0, ns = 0, stag = 0;
        double prev = INFINITY;
    };
    std::vector<St> s(L.n);
    for (auto& x : s) x.extra = grad ? 1 : 0;
    for (int it = 1; it <= 100; ++it) {
        SrcList A{}, B{};   // inverse-based and inverse-free steps this round
        for (int e = 0; e < L.n; ++e) {
            if (s[e].done) continue;
            SrcList& T = s[e].ns ? B : A;
            T.slot[T.n] = L.slot[e];
            T.src[T.n] = e;   // back-reference to the entry
            T.k[T.n] = L.k[e];
            T.flag[T.n] = s[e].scaling;
            ++T.n;
        }
        if (A.n == 0 && B.n == 0) break;
        SrcList R{};   // inverse-based entries close enough to test |I - X^2| afterwards
        for (int a = 0; a < A.n; ++a)
            if (s[A.src[a]].prev < kResidCheck) {
                R.slot[R.n] = A.slot[a];
                R.src[R.n] = A.src[a];
                R.k[R.n] = A.k[a];
                R.flag[R.n] = A.flag[a];
                ++R.n;
            }
        if (A.n) tslov::dense_newton_step(A, grad, choose_nb(c, A.k[0]), c->lds_max, w, c->st, tridiag_start && it == 1);
        if (R.n) tslov::dense_residual(R, w, c->st);
        if (B.n) tslov::dense_ns_step(B, grad, w, c->st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(c->host_part, w.delta, (size_t)4 * c->dslots * sizeof(double), hipMemcpyDeviceToHost,
                              c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        for (const SrcList* T : {&A, &B})
            for (int a = 0; a < T->n; ++a) {
                St& x = s[T->src[a]];
                x.it = it;
                const double* dl = c->host_part + 4 * T->slot[a];
                const double delta = std::sqrt(dl[0] / dl[1]);
                if (!std::isfinite(delta))
                    return fail(TSLOV_ERR_SIGN_UNDEFINED, "projected matrix is singular or its sign is undefined");
                if (x.ns && delta > x.prev) {   // not contracting: back to inverse-based steps
                    x.ns = 0;
                    x.prev = delta;
                    continue;
                }
                const bool tested = T == &A && x.prev < kResidCheck;   // residual taken this round
                if (delta < kNsSwitch || (tested && std::sqrt(dl[2]) < kNsSafe)) {
                    x.scaling = 0;
                    x.ns = 1;
                }
                // quadratic convergence: once the step is below 1e-8 the new iterate's error
                // is at rounding level; stagnation above that also ends the iteration
                const bool conv = delta <= 1e-8 || (delta < 1e-6 && delta > 0.5 * x.prev);
                if (conv && delta > 1e-8) x.stag = 1;
                if (conv) {
                    if (x.extra) x.extra = 0;
                    else x.done = 1;
                }
                x.prev = delta;
            }
    }
    iters.assign(L.n, 0);
    for (int e = 0; e < L.n; ++e) {
        if (!s[e].done)
            return fail(TSLOV_ERR_SIGN_UNDEFINED,
                        "sign iteration of the projected matrix did not converge (eigenvalue near Re z = 0)");
        iters[e] = s[e].it;
    }
    if (stagnated) {
        stagnated->assign(L.n, 0);
        for (int e = 0; e < L.n; ++e) (*stagnated)[e] = s[e].stag;
    }
    return TSLOV_OK;
}

// sgn(T) (and the Frechet step) of every entry, coefficients c_j and adjoint seeds.
tslov_status dense_step(tslov_ctx* c, const SrcList& L, int grad, std::vector<int>& iters,
                        std::vector<int>* stagnated = nullptr) {
    DenseWork w;
    CHK(ensure_dense(c, c->slots, c->kcap, w));
    tslov::launch_dense_build(c->coef, L, grad, w, c->st);
    CHK(newton(c, L, grad, w, iters, 1, stagnated));   // X_0 = T_k is tridiagonal
    tslov::launch_dense_extract(c->coef, L, grad, w, c->st);
    HIPCHK(hipGetLastError());
    return TSLOV_OK;
}

// Nested projected-matrix step of a single entry (slot 0, k = k_used > m): sgn(T) e_1
// = T W^{1/2} e_1 with W = (T^2)^{-1} formed densely (banded inverse, one product),
// W^{1/2} e_1 from an inner two-sided Lanczos process of size m on W, and the
// inner principal square root from the Newton sign of [[0, T'], [I, 0]].  Leaves
// coef.c like dense_step.  iters: the inner Newton steps.
tslov_status nested_dense_step(tslov_ctx* c, const SrcList& L, int m, std::vector<int>& iters,
                               std::vector<int>* stagnated) {
    const int k = L.k[0];
    DenseWork w;
    CHK(ensure_dense(c, c->slots, c->kcap, w));
    tslov::launch_dense_build(c->coef, L, 0, w, c->st);            // X = T
    tslov::launch_tridiag_inverse(L, w, c->st);                    // Xinv = T^{-1}
    tslov::launch_dense_gemm(L, w, 3, 3, 4, c->st);                // Zt = T^{-2} = W
    tslov::nest_prepare(w, k, c->st);                              // Y2 = W^T
    const size_t nv = (size_t)k * m + 6 * (size_t)k + 2 * ((size_t)m + 2);
    CHK(ensure(c->nestbuf, nv * sizeof(ZD) + ((size_t)m + 2) * sizeof(double) + 8 * sizeof(int)));
    tslov::NestWork nw;
    nw.Vb = c->nestbuf.as<ZD>();
    nw.vec = nw.Vb + (size_t)k * m;
    nw.alpha = nw.vec + 6 * (size_t)k;
    nw.gamma = nw.alpha + m + 2;
    nw.beta = (double*)(nw.gamma + m + 2);
    nw.status = (int*)(nw.beta + m + 2);
    tslov::nest_init(nw, k, c->st);
    for (int j = 0; j < m; ++j) tslov::nest_step(w, nw, k, j, m, c->st);
    HIPCHK(hipGetLastError());
    int st[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(st, nw.status, sizeof(st), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (st[2]) return fail(TSLOV_ERR_BREAKDOWN, "serious breakdown of the inner Lanczos process at its step " +
                                                    std::to_string(st[1]));
    const int mu = st[1];
    DenseWork w2;
    CHK(ensure_dense(c, 1, 2 * mu, w2));
    tslov::nest_block(nw, w2, mu, c->st);
    const SrcList L2 = make_list({0}, {2 * mu});
    CHK(newton(c, L2, 0, w2, iters, 0, stagnated));
    tslov::nest_finish(nw, w2, c->coef, k, mu, c->st);
    HIPCHK(hipGetLastError());
    return TSLOV_OK;
}

// Two-sided Lanczos process of size k on B = [[H, dH], [0, H]] (float64, this
// context's links and mu) from the source (x1, x2) (canonical; x1 null: zero),
// y = |x| V sgn(T) e_1 in both halves into y1, y2 (canonical).
tslov_status block_tsl(tslov_ctx* c, const tslov::BlockTangent& t, const ZD* x1, const ZD* x2, int k, ZD* y1,
                       ZD* y2, EntryStatus& es) {
    const Geom& g = c->g;
    const size_t fe = c->field_elems();
    const int nb = tslov::blk_blocks(g);
    CHK(ensure(c->blk, ((size_t)14 + 2 * (size_t)k) * fe * sizeof(ZD) + (size_t)8 * nb * sizeof(double)));
    tslov::BlockFields f;
    ZD* base = c->blk.as<ZD>();
    for (int h = 0; h < 2; ++h) {
        f.x[h] = base + (0 + h) * fe;
        f.v[h] = base + (2 + h) * fe;
        f.w[h] = base + (4 + h) * fe;
        f.vp[h] = base + (6 + h) * fe;
        f.wp[h] = base + (8 + h) * fe;
        f.a[h] = base + (10 + h) * fe;
        f.b[h] = base + (12 + h) * fe;
        f.basis[h] = base + (14 + (size_t)h * k) * fe;
    }
    double* p0 = (double*)(base + (14 + 2 * (size_t)k) * fe);
    double* p1 = p0 + 4 * nb;
    CHK(ensure_work(c, 1, k, 0));
    if (x1) tslov::launch_spinor_to_soa<double>(x1, f.x[0], g, nullptr, c->st);
    else tslov::launch_zero((double*)f.x[0], 2 * fe, c->st);
    tslov::launch_spinor_to_soa<double>(x2, f.x[1], g, nullptr, c->st);
    std::vector<int> init(16, 0);
    HIPCHK(hipMemcpyAsync(c->coef.status, init.data(), init.size() * sizeof(int), hipMemcpyHostToDevice, c->st));
    tslov::launch_blk_start(f, g, c->coef, p0, c->st);
    const ZD* U = c->U64.as<ZD>();
    for (int j = 1; j <= k; ++j) {
        tslov::launch_apply<double, double>(U, f.v[0], f.a[0], g, c->kappa, c->mu, 0, 1, c->st);
        tslov::launch_apply<double, double>(U, f.v[1], f.a[1], g, c->kappa, c->mu, 0, 1, c->st);
        tslov::launch_apply<double, double>(U, f.w[0], f.b[0], g, c->kappa, -c->mu, 0, 1, c->st);
        tslov::launch_apply<double, double>(U, f.w[1], f.b[1], g, c->kappa, -c->mu, 0, 1, c->st);
        tslov::launch_blk_tangent(U, t, g, c->kappa, c->mu, f.v[1], f.a[0], f.w[0], f.b[1], c->st);
        tslov::launch_blk_step(f, g, c->coef, p0, p1, j, k, c->st);
    }
    HIPCHK(hipGetLastError());
    int st[16];
    double misc[16];
    HIPCHK(hipMemcpyAsync(st, c->coef.status, sizeof(st), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(misc, c->coef.misc, sizeof(misc), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (st[2] == 3) return fail(TSLOV_ERR_ARG, "the block source is not finite");
    es = EntryStatus();
    es.k_used = st[1];
    es.breakdown = st[2];
    es.step = st[3];
    es.norm_x = misc[0];
    if (es.breakdown == 2)
        return fail(TSLOV_ERR_BREAKDOWN, "serious breakdown of the block Lanczos process at step " +
                                             std::to_string(es.step));
    const size_t n12 = (size_t)12 * g.V;
    if (es.k_used == 0) {
        tslov::launch_zero((double*)y1, 2 * n12, c->st);
        tslov::launch_zero((double*)y2, 2 * n12, c->st);
        HIPCHK(hipStreamSynchronize(c->st));
        return TSLOV_OK;
    }
    const SrcList Ld = make_list({0}, {es.k_used});
    std::vector<int> iters, stag;
    CHK(dense_step(c, Ld, 0, iters, &stag));
    es.iters = iters[0];
    es.flags = stag[0] ? TSLOV_FLAG_SIGN_STAGNATED : 0;
    for (int h = 0; h < 2; ++h) {
        Work<double> wk{};
        wk.V = f.basis[h];
        wk.fe = fe;
        wk.kcap = k;
        wk.ring = 0;
        tslov::launch_assemble<double>(g, wk, Ld, c->coef, nullptr, 0, h ? y2 : y1, c->st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return TSLOV_OK;
}

tslov_status block_args(tslov_ctx* c, int nu, int site, const double* X, tslov::BlockTangent& t) {
    if (!X) return fail(TSLOV_ERR_ARG, "null argument");
    if (nu < 0 || nu > 3 || site < 0 || site >= c->g.V) return fail(TSLOV_ERR_ARG, "link out of range");
    t.nu = nu;
    t.site = site;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int r = 0; r < 2; ++r) {
                t.X[a][b][r] = X[(a * 3 + b) * 2 + r];
                if (!std::isfinite(t.X[a][b][r])) return fail(TSLOV_ERR_ARG, "X is not finite");
            }
    return TSLOV_OK;
}

// ---------------------------------------------------------------- backward
struct GradOut {
    ZD* dU = nullptr;        // [src][4][V][3][3] or null
    ZD* dpsi = nullptr;      // [src][V][4][3] or null
    double* jsum = nullptr;  // current estimator: [4][V] sum of U(1) projections
    ZD* y = nullptr;         // recompute mode: sgn(H) psi per source, assembled segment by segment
    int accumulate = 0;
    int ward = 0;            // compute the Ward check (needs psi)
    const ZD* psi = nullptr;
    double ward_max = 0.0, g_max = 0.0;
};

// Reverse pass and force contraction for every entry of L (k = k_used, decreasing).
// In recompute mode (c->ring) the steps run in segments of m from the top; each
// segment first regenerates its basis vectors by replaying the forward steps from
// its checkpoint, then runs its reverse steps and adds its force terms.
template <typename R, typename RL>
tslov_status backward(tslov_ctx* c, const SrcList& L, GradOut& out) {
    const Geom& g = c->g;
    const Work<R> wk = work<R>(c);
    const Z<RL>* U = links<RL>(c);
    const int kmax = L.k[0];
    const int m = c->ring ? c->ring_m : 0;
    if (m && out.ward) return fail(TSLOV_ERR_ARG, "the Ward check needs every Krylov vector stored");
    // force contraction split in chunks of j for parallelism; the split depends on
    // the lattice (and the segment) only, so a source's result does not depend on
    // the batch it shares a launch with
    const int nchunk = force_chunks(g.V);
    CHK(ensure(c->gpart, (size_t)c->slots * nchunk * 36 * g.ldv * sizeof(ZD)));
    int nlt = 0;   // entries with k_used > j form a prefix
    PairTuner tune(c, 1, L.n);
    auto reverse_step = [&](int j) {
        int neq_end = nlt;
        while (neq_end < L.n && L.k[neq_end] == j) ++neq_end;
        if (nlt > 0) {
            const SrcList Llt = prefix(L, nlt);
            tslov::launch_bwd_ra<R>(g, wk, Llt, c->coef, j, c->st);
            tune.before(nlt);
            tslov::launch_bwd_rb<R, RL>(U, g, c->kappa, c->mu, wk, Llt, c->coef, j, 0, tune.ns(nlt), c->st,
                                    TimedLaunch(c, 1).t);
            tune.after(nlt);
        }
        if (neq_end > nlt) {
            const SrcList Leq = range(L, nlt, neq_end);
            tslov::launch_bwd_rb<R, RL>(U, g, c->kappa, c->mu, wk, Leq, c->coef, j, 1, 1, c->st);
        }
        nlt = neq_end;
    };
    // entries with k_used >= j form a prefix
    auto reaching = [&](int j) {
        int n = 0;
        while (n < L.n && L.k[n] >= j) ++n;
        return prefix(L, n);
    };
    if (!m) {
        auto loop = [&]() -> tslov_status {
            nlt = 0;
            for (int j = kmax; j >= 1; --j) reverse_step(j);
            return TSLOV_OK;
        };
        if (graphs_usable(c) && !tune.active()) {
            LoopKey key;
            key.list(L).buffers(c, wk, U, 1);
            CHK(run_captured(c, c->gbwd, key, loop));
        } else {
            CHK(loop());
        }
        tslov::launch_force<R>(g, c->kappa, c->mu, wk, L, nchunk, c->gpart.as<ZD>(), c->st);
    } else {
        tslov::launch_zero(c->gpart.as<double>(), (size_t)c->slots * nchunk * 72 * g.ldv, c->st);
        for (int seg = n_segments(kmax, m) - 1; seg >= 0; --seg) {
            const int j0 = 1 + seg * m, j1 = std::min(j0 + m - 1, kmax);
            if (seg > 0) CHK(checkpoint<R>(c, reaching(j0), seg, j0, 1));
            for (int j = j0; j <= std::min(j1 + 1, kmax); ++j) {
                const SrcList Lr = reaching(j);
                tslov::launch_fwd_replay<R, RL>(U, g, c->kappa, c->mu, wk, Lr, c->coef, j, c->st);
                if (j <= j1) tslov::launch_recur_replay<R>(g, wk, Lr, c->coef, j, c->st);
            }
            // the segment's share of y = |x| sum_j c_j v_j while its vectors are in the ring
            if (out.y) tslov::launch_assemble<R>(g, wk, reaching(j0), c->coef, nullptr, 0, out.y, c->st, j0, j1);
            for (int j = j1; j >= j0; --j) reverse_step(j);
            tslov::launch_force<R>(g, c->kappa, c->mu, wk, reaching(j0), nchunk, c->gpart.as<ZD>(), c->st, j0, j1,
                                   1);
        }
    }
    if (out.dU) tslov::launch_force_reduce(g, c->gpart.as<ZD>(), nchunk, L, c->antiperiodic, out.dU, c->st);
    double* gsrc = nullptr;
    if (out.ward) {
        CHK(ensure(c->gsrc, (size_t)c->slots * 4 * g.ldv * sizeof(double)));
        gsrc = c->gsrc.as<double>();
    }
    if (out.jsum)
        tslov::launch_force_current(g, c->gpart.as<ZD>(), nchunk, L, c->U64.as<ZD>(), gsrc, out.jsum,
                                    out.accumulate, c->st);
    if (out.dpsi) tslov::launch_source_grad<R>(g, wk, L, c->coef, out.dpsi, c->st);
    if (out.ward) {
        // per-entry y and dpsi in entry order
        const size_t n12 = (size_t)12 * g.V;
        CHK(ensure(c->bout, (size_t)2 * L.n * n12 * sizeof(ZD)));
        ZD* y = c->bout.as<ZD>();
        ZD* dp = y + L.n * n12;
        SrcList Le = L;
        for (int e = 0; e < L.n; ++e) Le.src[e] = e;
        tslov::launch_assemble<R>(g, wk, Le, c->coef, nullptr, 0, y, c->st);
        tslov::launch_source_grad<R>(g, wk, Le, c->coef, dp, c->st);
        const int nb = c->nblk();
        CHK(ensure(c->wardp, (size_t)L.n * nb * 2 * sizeof(double)));
        CHK(ensure_host_part(c, 2 * L.n * nb));
        tslov::launch_ward(g, gsrc, L, out.psi, y, dp, c->wardp.as<double>(), c->st);
        HIPCHK(hipMemcpyAsync(c->host_part, c->wardp.p, (size_t)L.n * nb * 2 * sizeof(double), hipMemcpyDeviceToHost,
                              c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        for (int i = 0; i < L.n * nb; ++i) {
            out.ward_max = std::max(out.ward_max, c->host_part[2 * i]);
            out.g_max = std::max(out.g_max, c->host_part[2 * i + 1]);
        }
    }
    HIPCHK(hipGetLastError());
    return TSLOV_OK;
}

tslov_status check_common(tslov_ctx* c, int k, const tslov_deflation* defl) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (!c->links_set) return fail(TSLOV_ERR_ARG, "links not set (call tslov_set_links first)");
    if (k < 1 || k > kMaxK) return fail(TSLOV_ERR_ARG, "k must be in [1, 1024]");
    if (defl && (defl->l < 0 || defl->l > kMaxDeflSet)) return fail(TSLOV_ERR_ARG, "deflation size must be in [0, 256]");
    return TSLOV_OK;
}

// Deflation set: validated on the host, signs copied to the device.
struct DeflSet {
    int l = 0;
    const ZD* R = nullptr;
    const ZD* L = nullptr;
    ZD* c = nullptr;
    double* sgn = nullptr;
    double* part = nullptr;
};

tslov_status prepare_defl(tslov_ctx* c, const tslov_deflation* defl, DeflSet& d) {
    d = DeflSet();
    if (!defl || defl->l == 0) return TSLOV_OK;
    if (defl->l < 0 || defl->l > kMaxDeflSet) return fail(TSLOV_ERR_ARG, "deflation size must be in [0, 256]");
    if (!defl->R || !defl->L || !defl->lambda) return fail(TSLOV_ERR_ARG, "deflation needs R, L and lambda");
    const int l = defl->l;
    std::vector<double> sg(l);
    double scale = 0.0;
    for (int i = 0; i < l; ++i) scale = std::max(scale, std::hypot(defl->lambda[2 * i], defl->lambda[2 * i + 1]));
    for (int i = 0; i < l; ++i) {
        const double re = defl->lambda[2 * i];
        if (!(std::fabs(re) > 1e-12 * scale)) return fail(TSLOV_ERR_SIGN_UNDEFINED, "deflated eigenvalue on Re z = 0");
        sg[i] = re > 0 ? 1.0 : -1.0;
    }
    const int nb = c->nblk();
    CHK(ensure(c->deflw, (size_t)l * sizeof(ZD) + (size_t)l * sizeof(double) + (size_t)nb * 2 * l * sizeof(double)));
    d.l = l;
    d.R = (const ZD*)defl->R;
    d.L = (const ZD*)defl->L;
    d.c = c->deflw.as<ZD>();
    d.sgn = (double*)(d.c + l);
    d.part = d.sgn + l;
    HIPCHK(hipMemcpyAsync(d.sgn, sg.data(), (size_t)l * sizeof(double), hipMemcpyHostToDevice, c->st));
    return TSLOV_OK;
}

// Canonical spinor buffers of a context: 0 projected source, 1 source gradient,
// 2 partial result (deflation); 3, 4 first and second result of the error
// estimate; 5 g5 eta of the overlap derivative; 6, 7 the second block-matrix
// result of the block error estimate.
constexpr int kCanonBufs = 8;
ZD* canon_buf(tslov_ctx* c, int i) { return c->canon.as<ZD>() + (size_t)i * 12 * c->g.V; }

void fill_info(tslov_info* info, const EntryStatus& s, const double* ms) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->k_used = s.k_used;
    info->breakdown = s.breakdown;
    info->newton_iters = s.iters;
    info->cg_iters = s.cg_iters;
    info->flags = s.flags;
    info->norm_x = s.norm_x;
    info->min_abs_re_ritz = s.k_used > 0 ? s.ritz.min_abs_re : NAN;
    info->norm_T = s.k_used > 0 ? s.ritz.norm_T : NAN;
    info->biorth_err = s.biorth;
    info->eps_A = s.eps_A;
    for (int i = 0; i < 6; ++i) info->ms[i] = ms[i];
}

// Flags of an entry after its dense step: Newton stagnation, an unsettled Ritz
// solve and (derivative calls) the float32 Krylov vectors of TSLOV_MIXED.
int entry_flags(const tslov_ctx* c, const EntryStatus& s, int stagnated, int grad) {
    int f = 0;
    if (stagnated) f |= TSLOV_FLAG_SIGN_STAGNATED;
    if (s.k_used > 0 && s.ritz.sweeps < 0) f |= TSLOV_FLAG_RITZ_UNSETTLED;
    if (grad && c->precision == TSLOV_MIXED) f |= TSLOV_FLAG_GRAD_FP32_VECTORS;
    return f;
}

tslov_status sign_dispatch(tslov_ctx* c, const void* psi, void* out, int k, const tslov_deflation* defl,
                           tslov_info* info, int overlap, int want_eps = 0);

// eps_A = |TSL(y) - psi| / (2 |psi|) for the first result y (Sec. 4.1 eq. error_est):
// a fresh two-sided Lanczos process with source y, the same k and deflation.  y may
// sit in canonical buffer 3; z takes buffer 4.
tslov_status error_of(tslov_ctx* c, const ZD* psi, const ZD* y, int k, const tslov_deflation* defl, double* eps) {
    const size_t n = (size_t)12 * c->g.V;
    CHK(ensure(c->canon, (size_t)kCanonBufs * n * sizeof(ZD)));
    ZD* z = canon_buf(c, 4);
    CHK(sign_dispatch(c, y, z, k, defl, nullptr, 0, 0));
    CHK(ensure_host_part(c, 2048));
    double* part = c->part.as<double>() + 2 * c->pstride();
    const int nb = tslov::launch_diff_norm(z, psi, n, part, c->st);
    HIPCHK(hipMemcpyAsync(c->host_part, part, (size_t)2 * nb * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    double dif = 0.0, nrm = 0.0;
    for (int i = 0; i < nb; ++i) {
        dif += c->host_part[2 * i];
        nrm += c->host_part[2 * i + 1];
    }
    // sgn(0) = 0 is exact: a zero source has no error
    *eps = nrm > 0.0 ? std::sqrt(dif / nrm) / 2.0 : 0.0;
    return TSLOV_OK;
}

// out = [psi +] g5^{overlap} sgn(H) psi by TSL, with optional deflation; with
// want_eps also eps_A into info (the sign itself then also goes to canonical
// buffer 3 when out holds the overlap).
template <typename R, typename RL>
tslov_status sign_impl(tslov_ctx* c, const void* psi_in, void* out, int k, const tslov_deflation* defl,
                       tslov_info* info, int overlap, int want_eps) {
    const double t0 = now_ms();
    DeflSet d;
    CHK(prepare_defl(c, defl, d));
    const ZD* psi = (const ZD*)psi_in;
    const ZD* src = psi;
    CHK(ensure(c->canon, (size_t)kCanonBufs * 12 * c->g.V * sizeof(ZD)));
    if (d.l) {
        tslov::launch_defl_coeffs(d.L, psi, c->g.V, d.l, d.part, d.c, c->st);
        tslov::launch_defl_project(d.R, psi, d.c, c->g.V, d.l, canon_buf(c, 0), c->st);
        src = canon_buf(c, 0);
    }
    CHK(ensure_work(c, 1, k, 0));
    const SrcList L = make_list({0}, {k});
    std::vector<EntryStatus> es;
    RitzJobs jobs;
    CHK((forward<R, RL>(c, L, src, nullptr, 0, es, &jobs)));
    if (es[0].breakdown == 2)
        return fail(TSLOV_ERR_BREAKDOWN, "serious Lanczos breakdown at step " + std::to_string(es[0].step));
    const double t1 = now_ms();
    const int k_used = es[0].k_used;
    SrcList Ld = make_list({0}, {k_used});
    std::vector<int> stag(1, 0);
    if (k_used > 0) {
        std::vector<int> iters;
        if (c->nest_m > 0 && c->nest_m < k_used) CHK(nested_dense_step(c, Ld, c->nest_m, iters, &stag));
        else CHK(dense_step(c, Ld, 0, iters, &stag));
        es[0].iters = iters[0];
    }
    const double t2 = now_ms();
    const Work<R> wk = work<R>(c);
    // y alone (no psi added) where the overlap is asked for and eps_A needs the sign
    ZD* ysign = (want_eps && overlap) ? canon_buf(c, 3) : nullptr;
    for (int pass = 0; pass < (ysign ? 2 : 1); ++pass) {
        const int ov = pass == 0 ? overlap : 0;
        ZD* o = pass == 0 ? (ZD*)out : ysign;
        if (d.l) {
            ZD* yp = nullptr;
            if (k_used > 0) {
                yp = canon_buf(c, 1);
                tslov::launch_assemble<R>(c->g, wk, Ld, c->coef, nullptr, 0, yp, c->st);
            }
            tslov::launch_defl_finish(d.R, d.c, d.sgn, yp, psi, c->g.V, d.l, ov, o, c->st);
        } else if (k_used > 0) {
            tslov::launch_assemble<R>(c->g, wk, Ld, c->coef, psi, ov, o, c->st);
        } else {
            tslov::launch_defl_finish(nullptr, nullptr, nullptr, nullptr, psi, c->g.V, 0, ov, o, c->st);
        }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    jobs.join();
    es[0].ritz = jobs.out[0];
    es[0].flags = entry_flags(c, es[0], stag[0], 0);
    CHK(check_ritz(es[0]));
    const double t3 = now_ms();
    if (want_eps) CHK(error_of(c, psi, ysign ? ysign : (const ZD*)out, k, defl, &es[0].eps_A));
    const double t4 = now_ms();
    const double ms[6] = {t1 - t0, t2 - t1, t3 - t2, 0.0, t4 - t3, t4 - t0};
    fill_info(info, es[0], ms);
    return TSLOV_OK;
}

// Batched S_s = Re <eta_s | TSL(psi_s)> and its link derivative for nsrc sources
// (canonical arrays indexed by source).  Sources are processed in groups of
// decreasing Krylov size that fit the device memory.
struct BatchRequest {
    int nsrc = 0;
    int recompute = 0;         // segment length of the Krylov-vector recompute (0: all stored)
    const ZD* eta = nullptr;   // null with eta_g5: eta = g5 psi
    int eta_g5 = 0;
    const ZD* psi = nullptr;
    const int* k = nullptr;
    double* S_out = nullptr;
    ZD* dU = nullptr;
    ZD* dpsi = nullptr;
    ZD* y = nullptr;           // sgn(H) psi per source (canonical, nullable)
    double* jsum = nullptr;
    int ward = 0;
    tslov_info* infos = nullptr;
    double ward_max = 0.0, g_max = 0.0;
};

template <typename R, typename RL>
tslov_status grad_batched(tslov_ctx* c, BatchRequest& q) {
    const double t0 = now_ms();
    std::vector<int> order(q.nsrc);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return q.k[a] > q.k[b]; });
    const size_t n12 = (size_t)12 * c->g.V;
    int first_group = 1;
    std::string broken;
    size_t pos = 0;
    while (pos < order.size()) {
        const int kcap = q.k[order[pos]];
        const int cap = group_size(c, kcap, 1, q.recompute, (int)(order.size() - pos));
        std::vector<int> src(order.begin() + pos, order.begin() + pos + cap), ks(cap);
        for (int e = 0; e < cap; ++e) ks[e] = q.k[src[e]];
        pos += cap;
        CHK(ensure_work(c, cap, kcap, 1, q.recompute));
        const double tg0 = now_ms();
        const SrcList L = make_list(src, ks);
        std::vector<EntryStatus> es;
        RitzJobs jobs;
        CHK((forward<R, RL>(c, L, q.psi, q.eta_g5 ? q.psi : q.eta, q.eta_g5, es, &jobs)));
        const double tg1 = now_ms();
        // entries that go on to the derivative, in decreasing k_used
        std::vector<int> live;
        for (int e = 0; e < cap; ++e) {
            const int s = src[e];
            if (es[e].breakdown == 2) {
                broken += (broken.empty() ? "" : ", ") + std::to_string(s) + " (step " + std::to_string(es[e].step) + ")";
                continue;
            }
            if (es[e].k_used == 0) {   // zero source: S = 0 and every derivative vanishes
                if (q.dU) tslov::launch_zero((double*)(q.dU + (size_t)s * 36 * c->g.V), (size_t)72 * c->g.V, c->st);
                if (q.dpsi) tslov::launch_zero((double*)(q.dpsi + (size_t)s * n12), 2 * n12, c->st);
                if (q.y) tslov::launch_zero((double*)(q.y + (size_t)s * n12), 2 * n12, c->st);
                if (q.S_out) q.S_out[s] = 0.0;
                continue;
            }
            live.push_back(e);
        }
        std::stable_sort(live.begin(), live.end(), [&](int a, int b) { return es[a].k_used > es[b].k_used; });
        SrcList Ld{};
        Ld.n = (int)live.size();
        for (int i = 0; i < Ld.n; ++i) {
            Ld.slot[i] = L.slot[live[i]];
            Ld.src[i] = L.src[live[i]];
            Ld.k[i] = es[live[i]].k_used;
        }
        std::vector<int> iters, stag;
        double tg2 = now_ms(), tg3 = tg2;
        if (Ld.n > 0) {
            CHK(dense_step(c, Ld, 1, iters, &stag));
            tg2 = now_ms();
            // with every vector stored y is assembled here; in recompute mode the reverse
            // pass assembles it segment by segment from the regenerated vectors
            if (q.y && !c->ring) tslov::launch_assemble<R>(c->g, work<R>(c), Ld, c->coef, nullptr, 0, q.y, c->st);
            GradOut go;
            go.y = c->ring ? q.y : nullptr;
            go.dU = q.dU;
            go.dpsi = q.dpsi;
            go.jsum = q.jsum;
            go.accumulate = first_group ? 0 : 1;
            go.ward = q.ward;
            go.psi = q.psi;
            CHK((backward<R, RL>(c, Ld, go)));
            q.ward_max = std::max(q.ward_max, go.ward_max);
            q.g_max = std::max(q.g_max, go.g_max);
            first_group = 0;
            std::vector<double> misc((size_t)16 * cap);
            HIPCHK(hipMemcpyAsync(misc.data(), c->coef.misc, misc.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  c->st));
            HIPCHK(hipStreamSynchronize(c->st));
            tg3 = now_ms();
            for (int i = 0; i < Ld.n; ++i) {
                const int e = live[i];
                es[e].iters = iters[i];
                es[e].flags = stag[i] ? TSLOV_FLAG_SIGN_STAGNATED : 0;
                es[e].S = misc[(size_t)16 * L.slot[e] + 1];
                if (q.S_out) q.S_out[src[e]] = es[e].S;
            }
        } else if (q.jsum && first_group) {
            tslov::launch_zero(q.jsum, (size_t)4 * c->g.V, c->st);
            first_group = 0;
        }
        HIPCHK(hipStreamSynchronize(c->st));
        jobs.join();
        for (int e = 0; e < cap; ++e) {
            es[e].ritz = jobs.out[e];
            es[e].flags = entry_flags(c, es[e], es[e].flags & TSLOV_FLAG_SIGN_STAGNATED, 1);
        }
        const double ms[6] = {tg1 - tg0, tg2 - tg1, 0.0, tg3 - tg2, 0.0, tg3 - tg0};
        if (q.infos)
            for (int e = 0; e < cap; ++e) fill_info(&q.infos[src[e]], es[e], ms);
        for (int e = 0; e < cap; ++e)
            if (es[e].breakdown != 2) CHK(check_ritz(es[e]));
    }
    if (q.jsum && first_group) tslov::launch_zero(q.jsum, (size_t)4 * c->g.V, c->st);
    HIPCHK(hipStreamSynchronize(c->st));
    (void)t0;
    if (!broken.empty()) return fail(TSLOV_ERR_BREAKDOWN, "serious Lanczos breakdown for source(s) " + broken);
    return TSLOV_OK;
}

tslov_status sign_dispatch(tslov_ctx* c, const void* psi, void* out, int k, const tslov_deflation* defl,
                           tslov_info* info, int overlap, int want_eps) {
    switch (c->precision) {
        case TSLOV_MIXED: return sign_impl<float, float>(c, psi, out, k, defl, info, overlap, want_eps);
        case TSLOV_FP32_LINKS: return sign_impl<double, float>(c, psi, out, k, defl, info, overlap, want_eps);
        default: return sign_impl<double, double>(c, psi, out, k, defl, info, overlap, want_eps);
    }
}

static tslov_status run_batched(tslov_ctx* c, BatchRequest& q) {
    switch (c->precision) {
        case TSLOV_MIXED: return grad_batched<float, float>(c, q);
        case TSLOV_FP32_LINKS: return grad_batched<double, float>(c, q);
        default: return grad_batched<double, double>(c, q);
    }
}

constexpr double kCgTol = 1e-13;     // relative residual of the shifted solves
constexpr int kCgMaxIter = 100000;
constexpr int kCgCheckEvery = 8;

// Workspace and per-system scalars of nr shifted systems (sigma_e - H(m_e mu)) x = b.
tslov_status cg_setup(tslov_ctx* c, int nr, const ZD* sigma, const double* msign, tslov::CgWork& cw) {
    const int ps = c->pstride();
    CHK(ensure(c->cgf, (size_t)nr * tslov::kCgFields * c->field_elems() * sizeof(ZD)));
    CHK(ensure(c->cgp, (size_t)nr * 4 * ps * sizeof(double)));
    CHK(ensure(c->cgs, (size_t)nr * sizeof(tslov::CgRhs)));
    cw.f = c->cgf.as<ZD>();
    cw.part = c->cgp.as<double>();
    cw.st = c->cgs.as<tslov::CgRhs>();
    cw.fe = c->field_elems();
    cw.pstride = ps;
    cw.op = c->cg_op;
    std::vector<tslov::CgRhs> st0(nr);
    for (int e = 0; e < nr; ++e) {
        st0[e] = tslov::CgRhs{};
        st0[e].sigma = sigma[e];
        st0[e].msign = msign[e];
    }
    HIPCHK(hipMemcpyAsync(cw.st, st0.data(), nr * sizeof(tslov::CgRhs), hipMemcpyHostToDevice, c->st));
    return TSLOV_OK;
}

// Conjugate gradients on the normal equations of the nr systems whose right-hand sides
// are loaded (r = b, x = 0, |b|^2 set): all in lockstep, each frozen once its residual
// is below kCgTol |b|; the convergence flags are read every kCgCheckEvery iterations.
tslov_status cg_solve(tslov_ctx* c, int nr, const tslov::CgWork& cw, int* iters) {
    const ZD* U = c->U64.as<ZD>();
    tslov::launch_cg_start(U, c->g, c->kappa, c->mu, nr, cw, c->st);
    int it = 0, all_done = 0;
    std::vector<tslov::CgRhs> sh(nr);
    for (; it < kCgMaxIter && !all_done; ++it) {
        const int check = (it % kCgCheckEvery) == kCgCheckEvery - 1;
        tslov::launch_cg_iteration(U, c->g, c->kappa, c->mu, nr, it, check, kCgTol, cw, c->st);
        if (check) {
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(sh.data(), cw.st, nr * sizeof(tslov::CgRhs), hipMemcpyDeviceToHost, c->st));
            HIPCHK(hipStreamSynchronize(c->st));
            all_done = 1;
            for (int e = 0; e < nr; ++e) all_done &= sh[e].done;
        }
    }
    *iters = it;
    if (!all_done) return fail(TSLOV_ERR_NOT_CONVERGED, "shifted solves of the eigenpair derivative did not converge");
    return TSLOV_OK;
}

// Derivative of the deflated S = Re eta^H [sum_i s_i Pi_i psi + TSL(P psi)], P = 1 - sum_i Pi_i,
// with the eigenpairs moving with U (reduced-resolvent solves; see solve.hip).
// Deflated derivative of nsrc sources at once (eta, psi, dU, dpsi, y: contiguous per
// source; k, S_out, infos: per source).  The TSL parts of all sources run as one
// batch; the 2l shifted systems of every source run as one batched CGNR of 2l nsrc
// systems, each system's arithmetic that of a solve of its own, so that a source gives
// the bits of its single-source call.
tslov_status deflated_grad_batched(tslov_ctx* c, int nsrc, const ZD* eta, const ZD* psi, const int* k,
                                   const tslov_deflation* defl, int recompute, double* S_out, ZD* dU, ZD* dpsi,
                                   ZD* y, tslov_info* infos) {
    const double t0 = now_ms();
    DeflSet d;
    CHK(prepare_defl(c, defl, d));
    const int l = d.l, V = c->g.V, nr = 2 * l;
    const size_t n12 = (size_t)12 * V, nfd = (size_t)12 * V * nsrc;
    const int nb = c->nblk();
    // canonical: projected sources, source gradients of the TSL part, TSL outputs (if y)
    CHK(ensure(c->deflb, (2 + (y ? 1 : 0)) * nfd * sizeof(ZD)));
    ZD* psip = c->deflb.as<ZD>();
    ZD* pbar = psip + nfd;
    ZD* ytsl = y ? pbar + nfd : nullptr;
    // per source: c (L^H psi), R^H eta, R^H psibar_p, q, -q (l each); dot partials
    CHK(ensure(c->deflx, (size_t)5 * l * nsrc * sizeof(ZD) + (size_t)nb * 2 * l * sizeof(double)));
    ZD* cd = c->deflx.as<ZD>();
    ZD* dRe = cd + (size_t)l * nsrc;
    ZD* dRp = dRe + (size_t)l * nsrc;
    ZD* qd = dRp + (size_t)l * nsrc;
    ZD* mqd = qd + (size_t)l * nsrc;
    double* xpart = (double*)(mqd + (size_t)l * nsrc);
    auto at = [&](const ZD* b, int s) { return b + (size_t)s * n12; };
    auto atm = [&](ZD* b, int s) { return b + (size_t)s * n12; };
    auto cof = [&](ZD* b, int s) { return b + (size_t)s * l; };
    for (int s = 0; s < nsrc; ++s) {
        tslov::launch_defl_coeffs(d.L, at(psi, s), V, l, xpart, cof(cd, s), c->st);            // c_i = L_i^H psi
        tslov::launch_defl_project(d.R, at(psi, s), cof(cd, s), V, l, atm(psip, s), c->st);    // psi_p = psi - R c
    }
    // TSL parts on the projected sources (link gradients into dU, source gradients into pbar)
    std::vector<double> S_tsl(nsrc, 0.0);
    BatchRequest q;
    q.nsrc = nsrc;
    q.eta = eta;
    q.psi = psip;
    q.k = k;
    q.S_out = S_tsl.data();
    q.dU = dU;
    q.dpsi = pbar;
    q.y = ytsl;
    q.infos = infos;
    q.recompute = recompute;
    CHK(run_batched(c, q));
    for (int s = 0; s < nsrc; ++s) {
        // y = TSL(psi_p) + sum_i s_i c_i R_i
        if (y) tslov::launch_defl_finish(d.R, cof(cd, s), d.sgn, at(ytsl, s), nullptr, V, l, 0, atm(y, s), c->st);
        tslov::launch_defl_coeffs(d.R, at(eta, s), V, l, xpart, cof(dRe, s), c->st);      // R_i^H eta
        tslov::launch_defl_coeffs(d.R, at(pbar, s), V, l, xpart, cof(dRp, s), c->st);     // R_i^H psibar_p
    }
    const size_t nl = (size_t)l * nsrc;
    std::vector<ZD> ch(nl), de(nl), dp(nl), qh(nl), mq(nl);
    std::vector<double> sg(l);
    HIPCHK(hipMemcpyAsync(ch.data(), cd, nl * sizeof(ZD), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(de.data(), dRe, nl * sizeof(ZD), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(dp.data(), dRp, nl * sizeof(ZD), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(sg.data(), d.sgn, l * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    std::vector<double> S(S_tsl);
    for (int s = 0; s < nsrc; ++s)
        for (int i = 0; i < l; ++i) {
            const size_t m = (size_t)s * l + i;
            qh[m] = ZD{sg[i] * de[m].re - dp[m].re, sg[i] * de[m].im - dp[m].im};   // R_i^H a_i
            mq[m] = ZD{-qh[m].re, -qh[m].im};
            S[s] += sg[i] * (de[m].re * ch[m].re + de[m].im * ch[m].im);         // Re conj(R_i^H eta) c_i
        }
    HIPCHK(hipMemcpyAsync(qd, qh.data(), nl * sizeof(ZD), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(mqd, mq.data(), nl * sizeof(ZD), hipMemcpyHostToDevice, c->st));
    // shifted solves of source s, systems 2 l s + e: e < l: (lambda_i - H) z = (1 - Pi_i) psi;
    // e >= l: (conj lambda_i - H^dag) z' = (1 - Pi_i^H) a_i
    const int nt = nr * nsrc;
    std::vector<ZD> sig(nt);
    std::vector<double> msg(nt);
    for (int s = 0; s < nsrc; ++s)
        for (int e = 0; e < nr; ++e) {
            const int i = e < l ? e : e - l;
            const double lr = defl->lambda[2 * i], li = defl->lambda[2 * i + 1];
            sig[(size_t)s * nr + e] = e < l ? ZD{lr, li} : ZD{lr, -li};
            msg[(size_t)s * nr + e] = e < l ? 1.0 : -1.0;
        }
    tslov::CgWork cw;
    CHK(cg_setup(c, nt, sig.data(), msg.data(), cw));
    auto view = [&](int s) {   // the source's 2l systems
        tslov::CgWork v = cw;
        v.f += (size_t)s * nr * tslov::kCgFields * cw.fe;
        v.part += (size_t)s * nr * 4 * cw.pstride;
        v.st += (size_t)s * nr;
        return v;
    };
    for (int s = 0; s < nsrc; ++s)
        tslov::launch_cg_rhs(c->g, at(psi, s), at(eta, s), at(pbar, s), d.R, d.L, cof(cd, s), cof(qd, s), d.sgn, l,
                             view(s), c->st);
    int it = 0;
    CHK(cg_solve(c, nt, cw, &it));
    for (int s = 0; s < nsrc; ++s) {
        tslov::launch_cg_finish(c->g, d.R, d.L, cof(cd, s), l, view(s), c->st);
        tslov::launch_defl_force(c->g, c->kappa, c->mu, d.R, d.L, cof(qd, s), l, view(s), c->antiperiodic,
                                 dU + (size_t)s * 36 * V, c->st);
        // source gradient: psibar = psibar_p + sum_i q_i L_i
        if (dpsi) tslov::launch_defl_project(d.L, at(pbar, s), cof(mqd, s), V, l, atm(dpsi, s), c->st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    for (int s = 0; s < nsrc; ++s) {
        if (S_out) S_out[s] = S[s];
        if (infos) {
            infos[s].cg_iters = it;
            infos[s].ms[4] = now_ms() - t0 - infos[s].ms[5];
            infos[s].ms[5] = now_ms() - t0;
        }
    }
    return TSLOV_OK;
}

tslov_status deflated_grad(tslov_ctx* c, const ZD* eta, const ZD* psi, int k, const tslov_deflation* defl,
                           int recompute, double* S_out, ZD* dU, ZD* dpsi, ZD* y, tslov_info* info) {
    return deflated_grad_batched(c, 1, eta, psi, &k, defl, recompute, S_out, dU, dpsi, y, info);
}

}  // namespace

// ===================================================================== C ABI
namespace {

// Chunk length of the t-march operator, picked on the first call by timing each
// candidate (best of three launches) on the call's own internal buffers: every
// candidate gives the same result, so the pick changes the time only.
template <typename R, typename RL>
tslov_status pick_apply_chunk(tslov_ctx* c, const Z<RL>* U, const Z<R>* a, Z<R>* b, double mu, int g5in, int g5out) {
    if (c->tm_T != 0) return TSLOV_OK;
    int cand[16];
    const int n = tslov::tmarch_chunks(c->g, cand, 16);
    if (n <= 1) {
        c->tm_T = n == 1 ? cand[0] : -1;
        return TSLOV_OK;
    }
    constexpr int kReps = 3;
    std::vector<hipEvent_t> ev((size_t)2 * n * kReps, nullptr);
    auto release_events = [&]() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            e = nullptr;
            release_events();
            return TSLOV_OK;   // no timing: the built-in choice stays
        }
    for (int r = 0; r < kReps; ++r)
        for (int i = 0; i < n; ++i) {
            const size_t x = (size_t)2 * (r * n + i);
            (void)hipEventRecord(ev[x], c->st);
            tslov::launch_apply<R, RL>(U, a, b, c->g, c->kappa, mu, g5in, g5out, c->st, tslov::Timing{}, cand[i]);
            (void)hipEventRecord(ev[x + 1], c->st);
        }
    const hipError_t es = hipEventSynchronize(ev.back());
    if (es == hipSuccess) {
        std::vector<float> best((size_t)n, 1e30f);
        for (int r = 0; r < kReps; ++r)
            for (int i = 0; i < n; ++i) {
                float ms = 0.0f;
                const size_t x = (size_t)2 * (r * n + i);
                if (hipEventElapsedTime(&ms, ev[x], ev[x + 1]) == hipSuccess) best[i] = std::min(best[i], ms);
            }
        int p = 0;
        for (int i = 1; i < n; ++i)
            if (best[i] < best[p]) p = i;
        c->tm_T = cand[p];
    }
    release_events();
    HIPCHK(es);
    return TSLOV_OK;
}

// The operator on canonical spinors: to the context's field layout, the stencil,
// and back.
// staging: the two SoA fields (the context's workspace, or the scratch array of
// the allocation-free entry point, which neither times launches nor picks the
// marching chunk length by timing: it takes the context's pick if one was made,
// else the built-in choice; every chunk length gives the same bits).
template <typename R, typename RL>
tslov_status apply_fields(tslov_ctx* c, const void* in, void* out, double mu, int g5in, int g5out, void* staging,
                          int no_alloc) {
    Z<R>* a = static_cast<Z<R>*>(staging);
    Z<R>* b = a + c->field_elems();
    const Z<RL>* U = links<RL>(c);
    tslov::launch_spinor_to_soa<R>((const ZD*)in, a, c->g, nullptr, c->st);
    if (!c->tm_T_forced && !no_alloc) CHK((pick_apply_chunk<R, RL>(c, U, a, b, mu, g5in, g5out)));
    tslov::launch_apply<R, RL>(U, a, b, c->g, c->kappa, mu, g5in, g5out, c->st,
                               no_alloc ? tslov::Timing{} : TimedLaunch(c, 2).t,
                               c->tm_T_forced ? c->tm_T_forced : std::max(c->tm_T, 0));
    tslov::launch_spinor_from_soa<R>(b, (ZD*)out, c->g, c->st);
    return TSLOV_OK;
}

}  // namespace

namespace {

// |v|^2 over n complex values (fixed-order block partials, host sum in block order).
tslov_status norm2_dev(tslov_ctx* c, const ZD* v, size_t n, double* out) {
    CHK(ensure_host_part(c, 8192));
    double* part = c->part.as<double>() + 2 * c->pstride();
    const int nb = tslov::launch_diff_norm(v, v, n, part, c->st);
    HIPCHK(hipMemcpyAsync(c->host_part, part, (size_t)2 * nb * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += c->host_part[2 * i + 1];
    *out = s;
    return TSLOV_OK;
}

// out = D_ov in (adjoint = 0) or D_ov^dag in (adjoint = 1) with the context's TSL sign of
// size k: D_ov = 1 + g5 sgn(H) (eq. overlap), and since sgn(H)^dag = sgn(H^dag) with
// H^dag = H(-mu), D_ov^dag = g5 D_ov(-mu) g5, the same process at -mu between two g5.
// tmp: a canonical scratch field.
tslov_status overlap_apply(tslov_ctx* c, const ZD* in, ZD* out, ZD* tmp, int k, int adjoint) {
    if (!adjoint) return sign_dispatch(c, in, out, k, nullptr, nullptr, 1, 0);
    const int V = c->g.V;
    tslov::launch_combine(nullptr, in, 1, V, tmp, c->st);
    const double mu = c->mu;
    c->mu = -mu;
    const tslov_status s = sign_dispatch(c, tmp, out, k, nullptr, nullptr, 1, 0);
    c->mu = mu;
    CHK(s);
    tslov::launch_combine(nullptr, out, 1, V, out, c->st);
    return TSLOV_OK;
}

// x with A x = b, A = D_ov (adjoint 0) or D_ov^dag (adjoint 1), by conjugate gradients on
// the normal equations A^dag A x = A^dag b, stopped at |b - A x| <= tol |b| (the TSL
// sign makes A an approximation, linear to its own accuracy).  Uses c->solvebuf.
tslov_status overlap_cgnr(tslov_ctx* c, const ZD* b, ZD* x, int k, int adjoint, double tol, int maxit, int* iters,
                          double* relres) {
    const size_t n = (size_t)12 * c->g.V;
    CHK(ensure(c->solvebuf, 5 * n * sizeof(ZD)));
    CHK(ensure_work(c, 1, k, 0));      // the sign's workspace, whose partial-sum array norm2_dev uses
    ZD* r = c->solvebuf.as<ZD>();
    ZD* z = r + n;
    ZD* p = z + n;
    ZD* w = p + n;
    ZD* tmp = w + n;
    double bb = 0.0, zz = 0.0, ww = 0.0, rr = 0.0;
    CHK(norm2_dev(c, b, n, &bb));
    tslov::launch_zero((double*)x, 2 * n, c->st);
    *iters = 0;
    *relres = 0.0;
    if (bb == 0.0) return TSLOV_OK;
    HIPCHK(hipMemcpyAsync(r, b, n * sizeof(ZD), hipMemcpyDeviceToDevice, c->st));
    CHK(overlap_apply(c, r, z, tmp, k, !adjoint));                  // z = A^dag r
    HIPCHK(hipMemcpyAsync(p, z, n * sizeof(ZD), hipMemcpyDeviceToDevice, c->st));
    CHK(norm2_dev(c, z, n, &zz));
    rr = bb;
    int it = 0;
    while (it < maxit && rr > tol * tol * bb && zz > 0.0) {
        CHK(overlap_apply(c, p, w, tmp, k, adjoint));               // w = A p
        CHK(norm2_dev(c, w, n, &ww));
        if (!(ww > 0.0)) break;
        const double alpha = zz / ww;
        tslov::launch_caxpy(p, alpha, x, n, c->st);
        tslov::launch_caxpy(w, -alpha, r, n, c->st);
        CHK(norm2_dev(c, r, n, &rr));
        ++it;
        if (rr <= tol * tol * bb) break;
        CHK(overlap_apply(c, r, z, tmp, k, !adjoint));              // z = A^dag r
        double zn = 0.0;
        CHK(norm2_dev(c, z, n, &zn));
        tslov::launch_cxpby(z, zn / zz, p, n, c->st);                // p = z + beta p
        zz = zn;
    }
    *iters = it;
    *relres = std::sqrt(rr / bb);
    if (*relres > tol) return fail(TSLOV_ERR_NOT_CONVERGED, "overlap solve did not reach its tolerance");
    return TSLOV_OK;
}

}  // namespace

namespace {

// eps_B of eq. bA_error_est for the tangent t and source (0, psi); ms_first (nullable)
// receives the wall time of the first block process.  Uses canonical buffers 3..7.
// out = dH in (canonical) for the link tangent t, through the float64 SoA fields f0, f1.
void apply_tangent(tslov_ctx* c, const tslov::BlockTangent& t, const ZD* in, ZD* out, ZD* f0, ZD* f1) {
    const Geom& g = c->g;
    tslov::launch_spinor_to_soa<double>(in, f0, g, nullptr, c->st);
    tslov::launch_zero((double*)f1, 2 * c->field_elems(), c->st);
    tslov::launch_blk_tangent(c->U64.as<ZD>(), t, g, c->kappa, c->mu, f0, f1, nullptr, nullptr, c->st);
    tslov::launch_spinor_from_soa<double>(f1, out, g, c->st);
}

// Deflated block-matrix process (App. E, eq. array_app_defl_1): with the l eigenpairs
// (lambda_i, R_i, L_i) of H (L^H R = 1) the 2l-dimensional invariant subspace of
// B = [[H, dH], [0, H]] spanned by (R_i, 0), (dR_i, R_i) is treated exactly:
//   c2_i = L_i^H x2,   c1_i = L_i^H x1 + <dL_i|x2>,
//   y = sum_i s_i [(R_i, 0) c1_i + (dR_i, R_i) c2_i] + TSL_k(B, Pbar x),
//   Pbar x = (x1 - sum_i (c1_i R_i + c2_i dR_i), x2 - sum_i c2_i R_i),
// s_i = sgn Re lambda_i; every coefficient from the input x (Pbar x then has no
// component along the deflated subspace).  The eigenvector derivatives (normalised
// <L_i|dR_i> = <dL_i|R_i> = 0, eq. c1i_3 and eq. dRi):
//   dR_i = sum_{j != i, j <= l} R_j (L_j^H dH R_i) / (lambda_i - lambda_j) + Q_i (lambda_i - H)^{-1} P_l dH R_i,
//   <dL_i|x2> = L_i^H dH [ sum_{j != i} R_j c2_j / (lambda_i - lambda_j) + Q_i (lambda_i - H)^{-1} P_l x2 ],
// P_l = 1 - sum_j R_j L_j^H, Q_i = 1 - R_i L_i^H.  The 2l singular consistent systems
// (lambda_i - H) z = P_l dH R_i and (lambda_i - H) z = P_l x2 go to one batched CGNR
// (the minimum-norm solution; Q_i removes its R_i component).
tslov_status block_tsl_deflated(tslov_ctx* c, const tslov::BlockTangent& t, const DeflSet& d, const double* lambda,
                                const ZD* x1, const ZD* x2, int k, ZD* y1, ZD* y2, EntryStatus& es) {
    const Geom& g = c->g;
    const int l = d.l, V = g.V, nb = c->nblk();
    const size_t n12 = (size_t)12 * V, fe = c->field_elems();
    // vectors: dHR[l], dR[l], Z[2l] (solutions), xk, p1, tmp, t1, t2 (canonical); f0, f1 (SoA);
    // scalars: M[l][l] (column i = L^H dH R_i), c1, c2, coefficient scratch (l each), one dot;
    // dot partials (nb x 2 l doubles)
    const size_t nvec = (size_t)4 * l + 5;
    CHK(ensure(c->bdefl, nvec * n12 * sizeof(ZD) + 2 * fe * sizeof(ZD) + ((size_t)l * l + 3 * (size_t)l + 1) * sizeof(ZD) +
                             (size_t)nb * 2 * l * sizeof(double)));
    ZD* base = c->bdefl.as<ZD>();
    ZD* dHR = base;
    ZD* dR = dHR + (size_t)l * n12;
    ZD* Z = dR + (size_t)l * n12;
    ZD* xk = Z + (size_t)2 * l * n12;
    ZD* p1 = xk + n12;
    ZD* tmp = p1 + n12;
    ZD* t1 = tmp + n12;
    ZD* t2 = t1 + n12;
    ZD* f0 = t2 + n12;
    ZD* f1 = f0 + fe;
    ZD* M = f1 + fe;
    ZD* c1 = M + (size_t)l * l;
    ZD* c2 = c1 + l;
    ZD* coef = c2 + l;
    ZD* dot = coef + l;
    double* part = (double*)(dot + 1);
    auto vec = [&](ZD* b, int i) { return b + (size_t)i * n12; };
    // dH R_i and M[., i] = L^H dH R_i
    for (int i = 0; i < l; ++i) {
        apply_tangent(c, t, d.R + (size_t)i * n12, vec(dHR, i), f0, f1);
        tslov::launch_defl_coeffs(d.L, vec(dHR, i), V, l, part, M + (size_t)i * l, c->st);
    }
    // c2 = L^H x2, xk = P_l x2; the right-hand sides P_l dH R_i in place
    tslov::launch_defl_coeffs(d.L, x2, V, l, part, c2, c->st);
    tslov::launch_defl_project(d.R, x2, c2, V, l, xk, c->st);
    for (int i = 0; i < l; ++i) tslov::launch_defl_project(d.R, vec(dHR, i), M + (size_t)i * l, V, l, vec(Z, i), c->st);
    std::vector<ZD> Mh((size_t)l * l), c2h(l);
    HIPCHK(hipMemcpyAsync(Mh.data(), M, Mh.size() * sizeof(ZD), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(c2h.data(), c2, l * sizeof(ZD), hipMemcpyDeviceToHost, c->st));
    // the 2l shifted systems: e < l with rhs P_l dH R_e (in Z[e]), e >= l with rhs xk
    const int nr = 2 * l;
    std::vector<ZD> sig(nr);
    std::vector<double> msg(nr, 1.0);
    for (int e = 0; e < nr; ++e) sig[e] = ZD{lambda[2 * (e % l)], lambda[2 * (e % l) + 1]};
    tslov::CgWork cw;
    CHK(cg_setup(c, nr, sig.data(), msg.data(), cw));
    tslov::launch_cg_load(g, Z, l, xk, nr, cw, c->st);
    int it = 0;
    CHK(cg_solve(c, nr, cw, &it));
    tslov::launch_cg_store(g, nr, cw, Z, c->st);
    // Q_i on each solution
    for (int e = 0; e < nr; ++e) {
        const int i = e % l;
        tslov::launch_defl_coeffs(d.L + (size_t)i * n12, vec(Z, e), V, 1, part, dot, c->st);
        tslov::launch_defl_project(d.R + (size_t)i * n12, vec(Z, e), dot, V, 1, vec(Z, e), c->st);
    }
    HIPCHK(hipStreamSynchronize(c->st));
    std::vector<ZD> ch(l);
    for (int i = 0; i < l; ++i) {
        const ZD li{lambda[2 * i], lambda[2 * i + 1]};
        // dR_i = Q_i z_i + sum_{j != i} R_j M[j][i] / (lambda_i - lambda_j)   (project with -coefficients)
        std::vector<ZD> a(l), b(l);
        for (int j = 0; j < l; ++j) {
            if (j == i) {
                a[j] = ZD{0.0, 0.0};
                b[j] = ZD{0.0, 0.0};
                continue;
            }
            const ZD dl{li.re - lambda[2 * j], li.im - lambda[2 * j + 1]};
            const double den = dl.re * dl.re + dl.im * dl.im;
            const ZD inv{dl.re / den, -dl.im / den};
            const ZD m = Mh[(size_t)i * l + j];
            a[j] = ZD{-(m.re * inv.re - m.im * inv.im), -(m.re * inv.im + m.im * inv.re)};
            b[j] = ZD{-(c2h[j].re * inv.re - c2h[j].im * inv.im), -(c2h[j].re * inv.im + c2h[j].im * inv.re)};
        }
        HIPCHK(hipMemcpyAsync(coef, a.data(), l * sizeof(ZD), hipMemcpyHostToDevice, c->st));
        tslov::launch_defl_project(d.R, vec(Z, i), coef, V, l, vec(dR, i), c->st);
        // v_i = Q_i w_i + sum_{j != i} R_j c2_j / (lambda_i - lambda_j);  c1_i = L_i^H (x1 + dH v_i)
        HIPCHK(hipMemcpyAsync(coef, b.data(), l * sizeof(ZD), hipMemcpyHostToDevice, c->st));
        tslov::launch_defl_project(d.R, vec(Z, l + i), coef, V, l, t1, c->st);
        apply_tangent(c, t, t1, t2, f0, f1);
        if (x1) tslov::launch_combine(x1, t2, 0, V, t2, c->st);   // t2 = x1 + dH v_i
        tslov::launch_defl_coeffs(d.L + (size_t)i * n12, t2, V, 1, part, c1 + i, c->st);
        HIPCHK(hipStreamSynchronize(c->st));   // a and b are reused by the next i
    }
    // Pbar x: p1 = x1 - R c1 - dR c2, p2 = xk
    if (x1) tslov::launch_defl_project(d.R, x1, c1, V, l, tmp, c->st);
    else {
        tslov::launch_zero((double*)p1, 2 * n12, c->st);
        tslov::launch_defl_project(d.R, p1, c1, V, l, tmp, c->st);
    }
    tslov::launch_defl_project(dR, tmp, c2, V, l, p1, c->st);
    CHK(block_tsl(c, t, p1, xk, k, y1, y2, es));
    // exact part: y1 += sum_i s_i (c1_i R_i + c2_i dR_i), y2 += sum_i s_i c2_i R_i
    tslov::launch_defl_finish(d.R, c1, d.sgn, y1, nullptr, V, l, 0, tmp, c->st);
    tslov::launch_defl_finish(dR, c2, d.sgn, tmp, nullptr, V, l, 0, y1, c->st);
    tslov::launch_defl_finish(d.R, c2, d.sgn, y2, nullptr, V, l, 0, tmp, c->st);
    HIPCHK(hipMemcpyAsync(y2, tmp, n12 * sizeof(ZD), hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    es.cg_iters = it;
    return TSLOV_OK;
}

// The block process with or without deflation.
tslov_status block_any(tslov_ctx* c, const tslov::BlockTangent& t, const DeflSet& d, const double* lambda,
                       const ZD* x1, const ZD* x2, int k, ZD* y1, ZD* y2, EntryStatus& es) {
    if (d.l > 0) return block_tsl_deflated(c, t, d, lambda, x1, x2, k, y1, y2, es);
    return block_tsl(c, t, x1, x2, k, y1, y2, es);
}

tslov_status block_eps(tslov_ctx* c, const tslov::BlockTangent& t, const ZD* psi, int k, double* eps_out,
                       double* ms_first, const DeflSet& d = DeflSet(), const double* lambda = nullptr) {
    const size_t n12 = (size_t)12 * c->g.V;
    CHK(ensure(c->canon, (size_t)kCanonBufs * n12 * sizeof(ZD)));
    ZD* y1 = canon_buf(c, 3);
    ZD* y2 = canon_buf(c, 4);
    ZD* z1 = canon_buf(c, 6);
    ZD* z2 = canon_buf(c, 7);
    ZD* zero = canon_buf(c, 5);
    EntryStatus es;
    HIPCHK(hipStreamSynchronize(c->st));
    const double t0 = now_ms();
    CHK(block_any(c, t, d, lambda, nullptr, psi, k, y1, y2, es));
    HIPCHK(hipStreamSynchronize(c->st));
    if (ms_first) *ms_first = now_ms() - t0;
    CHK(block_any(c, t, d, lambda, y1, y2, k, z1, z2, es));
    tslov::launch_zero((double*)zero, 2 * n12, c->st);
    CHK(ensure_host_part(c, 4096));
    double* part = c->part.as<double>() + 2 * c->pstride();
    double up = 0.0, lo = 0.0, nrm = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        const int nb = pass ? tslov::launch_diff_norm(z2, psi, n12, part, c->st)
                            : tslov::launch_diff_norm(zero, z1, n12, part, c->st);
        HIPCHK(hipMemcpyAsync(c->host_part, part, (size_t)2 * nb * sizeof(double), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        for (int i = 0; i < nb; ++i) {
            (pass ? lo : up) += c->host_part[2 * i];
            if (pass) nrm += c->host_part[2 * i + 1];
        }
    }
    *eps_out = nrm > 0.0 ? std::sqrt(up + lo) / (2.0 * std::sqrt(nrm)) : 0.0;
    return TSLOV_OK;
}

// One candidate of the tuning run on source psi: the error estimate and the wall
// time of the first approximation (its second run, so that allocation and first
// touch of a larger workspace do not count).  A candidate whose process breaks
// down or whose projected matrix has a Ritz value on the imaginary axis gets an
// infinite error.
tslov_status tune_candidate(tslov_ctx* c, const ZD* psi, int k, int k_inner, const tslov_deflation* defl,
                            const tslov::BlockTangent* t, double* eps, double* ms) {
    auto soft = [&](tslov_status s) {
        if (s == TSLOV_ERR_BREAKDOWN || s == TSLOV_ERR_SIGN_UNDEFINED) {
            *eps = INFINITY;
            *ms = NAN;
            return TSLOV_OK;
        }
        return s;
    };
    if (t) {
        DeflSet d;
        CHK(prepare_defl(c, defl, d));
        const double* lam = d.l ? defl->lambda : nullptr;
        double m0 = 0.0;
        tslov_status s = block_eps(c, *t, psi, k, eps, &m0, d, lam);
        if (s == TSLOV_OK) s = block_eps(c, *t, psi, k, eps, ms, d, lam);
        return soft(s);
    }
    const int keep = c->nest_m;
    c->nest_m = k_inner;
    ZD* y = canon_buf(c, 3);
    tslov_status s = sign_dispatch(c, psi, y, k, defl, nullptr, 0, 0);
    if (s == TSLOV_OK) {
        HIPCHK(hipStreamSynchronize(c->st));
        const double t0 = now_ms();
        s = sign_dispatch(c, psi, y, k, defl, nullptr, 0, 0);
        if (s == TSLOV_OK) {
            HIPCHK(hipStreamSynchronize(c->st));
            *ms = now_ms() - t0;
            s = error_of(c, psi, y, k, defl, eps);
        }
    }
    c->nest_m = keep;
    return soft(s);
}

}  // namespace

extern "C" {

const char* tslov_last_error(void) { return g_err.c_str(); }

tslov_status tslov_create(const tslov_lattice_desc* d, void* stream, tslov_ctx** out) {
    if (!d || !out) return fail(TSLOV_ERR_ARG, "null argument");
    *out = nullptr;
    for (int i = 0; i < 4; ++i)
        if (d->dims[i] < 2) return fail(TSLOV_ERR_ARG, "every lattice extent must be >= 2");
    if (d->precision != TSLOV_FP64 && d->precision != TSLOV_MIXED && d->precision != TSLOV_FP32_LINKS)
        return fail(TSLOV_ERR_ARG, "unknown precision");
    if (2.0 * d->mass + 8.0 == 0.0) return fail(TSLOV_ERR_ARG, "2*mass + 8 must be non-zero");
    const long long V = (long long)d->dims[0] * d->dims[1] * d->dims[2] * d->dims[3];
    if (V > (1LL << 26)) return fail(TSLOV_ERR_ARG, "lattice volume too large");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    char* scr = nullptr;
    CHK(scratch_address(dev, &scr));
    tslov_ctx* c = new tslov_ctx();
    c->device = dev;
    c->scratch = scr;
    c->lds_max = prop.sharedMemPerBlock ? prop.sharedMemPerBlock : 65536;
    c->g.nx = d->dims[0];
    c->g.ny = d->dims[1];
    c->g.nz = d->dims[2];
    c->g.nt = d->dims[3];
    c->g.V = (int)V;
    c->g.ldv = (int)((V + 63) / 64 * 64);
    c->kappa = 1.0 / (2.0 * d->mass + 8.0);
    c->mu = d->mu;
    c->antiperiodic = d->antiperiodic_t ? 1 : 0;
    c->precision = d->precision;
    c->st = (hipStream_t)stream;
    tslov_status s = ensure(c->U64, (size_t)36 * c->g.ldv * sizeof(ZD));
    if (s == TSLOV_OK && c->precision != TSLOV_FP64) s = ensure(c->U32, (size_t)36 * c->g.ldv * sizeof(Z<float>));
    if (s == TSLOV_OK) {
        int nwg = 0;
        const std::vector<int> map = site_block_order(c->g, nwg);
        s = ensure(c->sbmap, map.size() * sizeof(int));
        if (s == TSLOV_OK && hipMemcpy(c->sbmap.p, map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice) !=
                                 hipSuccess)
            s = fail(TSLOV_ERR_HIP, "copy of the site-block order failed");
        c->g.sbmap = c->sbmap.as<int>();
        c->g.nwg = nwg;
    }
    if (s != TSLOV_OK) {
        tslov_destroy(c);
        return s;
    }
    *out = c;
    return TSLOV_OK;
}

void tslov_destroy(tslov_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    for (Buf* b : {&c->trial, &c->solvebuf, &c->physbuf, &c->U64, &c->U32, &c->badflag, &c->nestbuf, &c->blk, &c->bdefl, &c->deflb, &c->curdefl, &c->sbmap, &c->opf, &c->basisV, &c->basisW, &c->basisA, &c->basisB, &c->abarS, &c->sbarS,
                   &c->fields, &c->part, &c->coefmem, &c->dense, &c->denseInt, &c->densePart, &c->denseDelta,
                   &c->gpart, &c->gsrc, &c->bout, &c->wardp, &c->canon, &c->deflw, &c->deflx, &c->cgf, &c->cgp,
                   &c->cgs, &c->ckpt})
        release(*b);
    c->gfwd.reset();
    c->gbwd.reset();
    if (c->host_part) (void)hipHostFree(c->host_part);
    for (auto& v : c->ev_used)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (auto e : c->ev_free) (void)hipEventDestroy(e);
    delete c;
}

tslov_status tslov_set_links(tslov_ctx* c, const void* U) {
    if (!c || !U) return fail(TSLOV_ERR_ARG, "null argument");
    CHK(ensure(c->badflag, sizeof(double)));
    tslov::launch_zero(c->badflag.as<double>(), 1, c->st);
    tslov::launch_links_to_soa((const ZD*)U, c->U64.as<ZD>(), c->precision != TSLOV_FP64 ? c->U32.as<Z<float>>() : nullptr,
                               c->g, c->antiperiodic, c->badflag.as<int>(), c->st);
    HIPCHK(hipGetLastError());
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, c->badflag.p, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    c->links_set = bad ? 0 : 1;
    if (bad) return fail(TSLOV_ERR_ARG, "the gauge field contains non-finite values");
    return TSLOV_OK;
}

static tslov_status apply_op(tslov_ctx* c, const void* in, void* out, double mu, int g5in, int g5out,
                             int no_alloc = 0) {
    if (!c || !in || !out) return fail(TSLOV_ERR_ARG, "null argument");
    if (!c->links_set) return fail(TSLOV_ERR_ARG, "links not set (call tslov_set_links first)");
    if (in == out) return fail(TSLOV_ERR_ARG, "in and out must not overlap");
    void* staging = nullptr;
    if (no_alloc) {
        if (2 * c->field_bytes() > kScratchBytes)
            return fail(TSLOV_ERR_ARG, "lattice too large for the allocation-free operator (" +
                                           std::to_string(2 * c->field_bytes()) + " bytes of staging, at most " +
                                           std::to_string(kScratchBytes) + ")");
        staging = c->scratch;
    } else {
        CHK(ensure(c->opf, 2 * c->field_bytes()));
        staging = c->opf.p;
    }
    switch (c->precision) {
        case TSLOV_MIXED: CHK((apply_fields<float, float>(c, in, out, mu, g5in, g5out, staging, no_alloc))); break;
        case TSLOV_FP32_LINKS:
            CHK((apply_fields<double, float>(c, in, out, mu, g5in, g5out, staging, no_alloc)));
            break;
        default: CHK((apply_fields<double, double>(c, in, out, mu, g5in, g5out, staging, no_alloc)));
    }
    HIPCHK(hipGetLastError());
    return TSLOV_OK;
}

tslov_status tslov_apply_dw(tslov_ctx* c, const void* in, void* out, int dagger) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    return dagger ? apply_op(c, in, out, -c->mu, 1, 1) : apply_op(c, in, out, c->mu, 0, 0);
}

tslov_status tslov_apply_h(tslov_ctx* c, const void* in, void* out, int dagger) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    return apply_op(c, in, out, dagger ? -c->mu : c->mu, 0, 1);
}

tslov_status tslov_apply_h_noalloc(tslov_ctx* c, const void* in, void* out, int dagger) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    return apply_op(c, in, out, dagger ? -c->mu : c->mu, 0, 1, 1);
}

tslov_status tslov_sign(tslov_ctx* c, const void* psi, void* out, int k, const tslov_deflation* defl,
                        tslov_info* info) {
    CHK(check_common(c, k, defl));
    if (!psi || !out) return fail(TSLOV_ERR_ARG, "null argument");
    if (psi == out) return fail(TSLOV_ERR_ARG, "psi and out must not overlap");
    return sign_dispatch(c, psi, out, k, defl, info, 0, (c->diag & TSLOV_DIAG_EPS_A) && info);
}

tslov_status tslov_overlap(tslov_ctx* c, const void* psi, void* out, int k, const tslov_deflation* defl,
                           tslov_info* info) {
    CHK(check_common(c, k, defl));
    if (!psi || !out) return fail(TSLOV_ERR_ARG, "null argument");
    if (psi == out) return fail(TSLOV_ERR_ARG, "psi and out must not overlap");
    return sign_dispatch(c, psi, out, k, defl, info, 1, (c->diag & TSLOV_DIAG_EPS_A) && info);
}

tslov_status tslov_sign_grad(tslov_ctx* c, const void* eta, const void* psi, int k, const tslov_deflation* defl,
                             int recompute_stride, double* S_out, void* dU_out, void* dpsi_out, void* y_out,
                             tslov_info* info) {
    CHK(check_common(c, k, defl));
    if (!eta || !psi || !dU_out) return fail(TSLOV_ERR_ARG, "null argument");
    if (recompute_stride < 0) return fail(TSLOV_ERR_ARG, "recompute_stride must be >= 0");
    if (y_out && (y_out == psi || y_out == eta)) return fail(TSLOV_ERR_ARG, "y_out must not overlap the inputs");
    const int want_eps = (c->diag & TSLOV_DIAG_EPS_A) && info;
    ZD* y = (ZD*)y_out;
    if (want_eps && !y) {
        CHK(ensure(c->canon, (size_t)kCanonBufs * 12 * c->g.V * sizeof(ZD)));
        y = canon_buf(c, 3);
    }
    if (defl && defl->l != 0) {
        CHK(deflated_grad(c, (const ZD*)eta, (const ZD*)psi, k, defl, recompute_stride, S_out, (ZD*)dU_out,
                          (ZD*)dpsi_out, y, info));
    } else {
        BatchRequest q;
        q.nsrc = 1;
        q.eta = (const ZD*)eta;
        q.psi = (const ZD*)psi;
        q.k = &k;
        q.S_out = S_out;
        q.dU = (ZD*)dU_out;
        q.dpsi = (ZD*)dpsi_out;
        q.y = y;
        q.infos = info;
        q.recompute = recompute_stride;
        CHK(run_batched(c, q));
    }
    if (want_eps) {
        const double t0 = now_ms();
        CHK(error_of(c, (const ZD*)psi, y, k, defl, &info->eps_A));
        info->ms[4] += now_ms() - t0;
        info->ms[5] += now_ms() - t0;
    }
    return TSLOV_OK;
}

tslov_status tslov_overlap_grad(tslov_ctx* c, const void* eta, const void* psi, int k, const tslov_deflation* defl,
                                int recompute_stride, double* S_out, void* dU_out, void* dpsi_out, void* dov_out,
                                tslov_info* info) {
    CHK(check_common(c, k, defl));
    if (!eta || !psi || !dU_out) return fail(TSLOV_ERR_ARG, "null argument");
    if (dov_out && (dov_out == psi || dov_out == eta)) return fail(TSLOV_ERR_ARG, "dov_out must not overlap the inputs");
    if (dpsi_out && (dpsi_out == psi || dpsi_out == eta)) return fail(TSLOV_ERR_ARG, "dpsi_out must not overlap the inputs");
    const int V = c->g.V;
    CHK(ensure(c->canon, (size_t)kCanonBufs * 12 * V * sizeof(ZD)));
    ZD* g5eta = canon_buf(c, 5);
    tslov::launch_combine(nullptr, (const ZD*)eta, 1, V, g5eta, c->st);
    // Re eta^H psi by the deflation dot kernels (one vector)
    CHK(ensure(c->deflx, (size_t)4 * sizeof(ZD) + (size_t)c->nblk() * 2 * sizeof(double)));
    ZD* dot = c->deflx.as<ZD>();
    tslov::launch_defl_coeffs((const ZD*)eta, (const ZD*)psi, V, 1, (double*)(dot + 4), dot, c->st);
    ZD hdot{0.0, 0.0};
    HIPCHK(hipMemcpyAsync(&hdot, dot, sizeof(ZD), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    double S = 0.0;
    CHK(tslov_sign_grad(c, g5eta, psi, k, defl, recompute_stride, &S, dU_out, dpsi_out, dov_out, info));
    if (dpsi_out) tslov::launch_combine((const ZD*)eta, (const ZD*)dpsi_out, 0, V, (ZD*)dpsi_out, c->st);
    if (dov_out) tslov::launch_combine((const ZD*)psi, (const ZD*)dov_out, 1, V, (ZD*)dov_out, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    if (S_out) *S_out = S + hdot.re;
    return TSLOV_OK;
}

tslov_status tslov_sign_grad_batched(tslov_ctx* c, int nsrc, const void* eta, const void* psi, const int* k,
                                     double* S_out, void* dU_out, void* dpsi_out, void* y_out, tslov_info* infos) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (!c->links_set) return fail(TSLOV_ERR_ARG, "links not set (call tslov_set_links first)");
    if (nsrc < 1 || nsrc > kMaxSources) return fail(TSLOV_ERR_ARG, "nsrc must be in [1, 2^20]");
    if (!eta || !psi || !k || !dU_out) return fail(TSLOV_ERR_ARG, "null argument");
    for (int s = 0; s < nsrc; ++s)
        if (k[s] < 1 || k[s] > kMaxK) return fail(TSLOV_ERR_ARG, "every k must be in [1, 1024]");
    BatchRequest q;
    q.nsrc = nsrc;
    q.eta = (const ZD*)eta;
    q.psi = (const ZD*)psi;
    q.k = k;
    q.S_out = S_out;
    q.dU = (ZD*)dU_out;
    q.dpsi = (ZD*)dpsi_out;
    q.y = (ZD*)y_out;
    q.infos = infos;
    return run_batched(c, q);
}

tslov_status tslov_sign_grad_batched_deflated(tslov_ctx* c, int nsrc, const void* eta, const void* psi, const int* k,
                                              const tslov_deflation* defl, double* S_out, void* dU_out,
                                              void* dpsi_out, void* y_out, tslov_info* infos) {
    if (!defl || defl->l == 0)
        return tslov_sign_grad_batched(c, nsrc, eta, psi, k, S_out, dU_out, dpsi_out, y_out, infos);
    CHK(check_common(c, 1, defl));
    if (nsrc < 1 || nsrc > kMaxSources) return fail(TSLOV_ERR_ARG, "nsrc must be in [1, 2^20]");
    if (!eta || !psi || !k || !dU_out) return fail(TSLOV_ERR_ARG, "null argument");
    for (int s = 0; s < nsrc; ++s)
        if (k[s] < 1 || k[s] > kMaxK) return fail(TSLOV_ERR_ARG, "every k must be in [1, 1024]");
    if (infos) std::memset(infos, 0, (size_t)nsrc * sizeof(tslov_info));
    return deflated_grad_batched(c, nsrc, (const ZD*)eta, (const ZD*)psi, k, defl, 0, S_out, (ZD*)dU_out,
                                 (ZD*)dpsi_out, (ZD*)y_out, infos);
}

tslov_status tslov_current_estimate(tslov_ctx* c, int nsrc, const void* xi, const int* k, double* j_out,
                                    double* div_out, double* tot_out, double* ward_out, tslov_info* infos) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (!c->links_set) return fail(TSLOV_ERR_ARG, "links not set (call tslov_set_links first)");
    if (nsrc < 1 || nsrc > kMaxSources) return fail(TSLOV_ERR_ARG, "nsrc must be in [1, 2^20]");
    if (!xi || !k || !j_out) return fail(TSLOV_ERR_ARG, "null argument");
    for (int s = 0; s < nsrc; ++s)
        if (k[s] < 1 || k[s] > kMaxK) return fail(TSLOV_ERR_ARG, "every k must be in [1, 1024]");
    BatchRequest q;
    q.nsrc = nsrc;
    q.eta_g5 = 1;
    q.psi = (const ZD*)xi;
    q.k = k;
    q.jsum = j_out;
    q.ward = ward_out ? 1 : 0;
    q.infos = infos;
    CHK(run_batched(c, q));
    tslov::launch_current_finish(c->g, j_out, 1.0 / nsrc, div_out, tot_out, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    if (ward_out) *ward_out = q.g_max > 0.0 ? q.ward_max / q.g_max : q.ward_max;
    return TSLOV_OK;
}

tslov_status tslov_current_estimate_deflated(tslov_ctx* c, int nsrc, const void* xi, const int* k,
                                             const tslov_deflation* defl, double* j_out, double* div_out,
                                             double* tot_out, double* ward_out, tslov_info* infos) {
    if (!defl || defl->l == 0) return tslov_current_estimate(c, nsrc, xi, k, j_out, div_out, tot_out, ward_out, infos);
    CHK(check_common(c, 1, defl));
    if (nsrc < 1 || nsrc > kMaxSources) return fail(TSLOV_ERR_ARG, "nsrc must be in [1, 2^20]");
    if (!xi || !k || !j_out) return fail(TSLOV_ERR_ARG, "null argument");
    for (int s = 0; s < nsrc; ++s)
        if (k[s] < 1 || k[s] > kMaxK) return fail(TSLOV_ERR_ARG, "every k must be in [1, 1024]");
    const Geom& g = c->g;
    const int V = g.V;
    const size_t n12 = (size_t)12 * V, nfd = n12 * nsrc;
    // eta_s = g5 xi_s, per-source dU, y and dpsi (the latter two for the Ward check)
    const int want_w = ward_out ? 1 : 0;
    CHK(ensure(c->curdefl, (nfd * (1 + 2 * want_w) + (size_t)nsrc * 36 * V) * sizeof(ZD) +
                               (want_w ? (size_t)nsrc * 4 * g.ldv * sizeof(double) : 0)));
    ZD* eta = c->curdefl.as<ZD>();
    ZD* dU = eta + nfd;
    ZD* y = want_w ? dU + (size_t)nsrc * 36 * V : nullptr;
    ZD* dp = want_w ? y + nfd : nullptr;
    double* gsrc = want_w ? (double*)(dp + nfd) : nullptr;
    const ZD* xs = (const ZD*)xi;
    for (int s = 0; s < nsrc; ++s) tslov::launch_g5_scale(xs + (size_t)s * n12, ZD{1.0, 0.0}, V, eta + (size_t)s * n12, c->st);
    if (infos) std::memset(infos, 0, (size_t)nsrc * sizeof(tslov_info));
    CHK(deflated_grad_batched(c, nsrc, eta, xs, k, defl, 0, nullptr, dU, dp, y, infos));
    tslov::launch_u1_projection(g, c->U64.as<ZD>(), dU, nsrc, c->antiperiodic, gsrc, j_out, 0, c->st);
    if (want_w) {
        // per-sample Ward residuals, in chunks of kMaxBatch entries
        double wmax = 0.0, gmax = 0.0;
        const int nb = c->nblk();
        for (int s0 = 0; s0 < nsrc; s0 += tslov::kMaxBatch) {
            const int n = std::min(nsrc - s0, tslov::kMaxBatch);
            SrcList L{};
            L.n = n;
            for (int e = 0; e < n; ++e) {
                L.slot[e] = e;
                L.src[e] = s0 + e;
                L.k[e] = k[s0 + e];
            }
            CHK(ensure(c->wardp, (size_t)n * nb * 2 * sizeof(double)));
            CHK(ensure_host_part(c, 2 * n * nb));
            tslov::launch_ward(g, gsrc + (size_t)s0 * 4 * g.ldv, L, xs, y + (size_t)s0 * n12, dp + (size_t)s0 * n12,
                               c->wardp.as<double>(), c->st);
            HIPCHK(hipMemcpyAsync(c->host_part, c->wardp.p, (size_t)n * nb * 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, c->st));
            HIPCHK(hipStreamSynchronize(c->st));
            for (int i = 0; i < n * nb; ++i) {
                wmax = std::max(wmax, c->host_part[2 * i]);
                gmax = std::max(gmax, c->host_part[2 * i + 1]);
            }
        }
        *ward_out = gmax > 0.0 ? wmax / gmax : wmax;
    }
    tslov::launch_current_finish(g, j_out, 1.0 / nsrc, div_out, tot_out, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return TSLOV_OK;
}

tslov_status tslov_overlap_solve(tslov_ctx* c, const void* b, void* x, int k, int adjoint, double tol, int maxit,
                                int* iters_out, double* relres_out) {
    CHK(check_common(c, k, nullptr));
    if (!b || !x) return fail(TSLOV_ERR_ARG, "null argument");
    if (b == x) return fail(TSLOV_ERR_ARG, "b and x must not overlap");
    if (!(tol > 0.0) || maxit < 1) return fail(TSLOV_ERR_ARG, "tol must be > 0 and maxit >= 1");
    int it = 0;
    double rel = 0.0;
    const tslov_status s = overlap_cgnr(c, (const ZD*)b, (ZD*)x, k, adjoint ? 1 : 0, tol, maxit, &it, &rel);
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = rel;
    return s;
}

tslov_status tslov_physical_current(tslov_ctx* c, int nsrc, const void* xi, int k, double tol, int maxit, double* j_out,
                                    double* div_out, double* tot_out, int* iters_out, double* relres_out) {
    CHK(check_common(c, k, nullptr));
    if (nsrc < 1 || nsrc > kMaxSources) return fail(TSLOV_ERR_ARG, "nsrc must be in [1, 2^20]");
    if (!xi || !j_out) return fail(TSLOV_ERR_ARG, "null argument");
    if (!(tol > 0.0) || maxit < 1) return fail(TSLOV_ERR_ARG, "tol must be > 0 and maxit >= 1");
    const int V = c->g.V;
    const size_t n = (size_t)12 * V;
    CHK(ensure(c->physbuf, 2 * (size_t)nsrc * n * sizeof(ZD)));
    ZD* chi = c->physbuf.as<ZD>();
    ZD* probe = chi + (size_t)nsrc * n;
    // chi_s = D_ov^{-dag} xi_s, so that xi_s^dag D_ov^{-1} = chi_s^dag
    for (int s = 0; s < nsrc; ++s) {
        int it = 0;
        double rel = 0.0;
        CHK(overlap_cgnr(c, (const ZD*)xi + (size_t)s * n, chi + (size_t)s * n, k, 1, tol, maxit, &it, &rel));
        if (iters_out) iters_out[s] = it;
        if (relres_out) relres_out[s] = rel;
    }
    // d/dTheta Re <eta|sgn(H)|xi> with eta = g5 chi gives Re chi^dag dD_ov/dTheta xi, and
    // with eta = i g5 chi its imaginary part; each summed over the sources by the batch
    std::vector<int> ks(nsrc, k);
    for (int part = 0; part < 2; ++part) {
        const ZD f = part ? ZD{0.0, 1.0} : ZD{1.0, 0.0};
        for (int s = 0; s < nsrc; ++s)
            tslov::launch_g5_scale(chi + (size_t)s * n, f, V, probe + (size_t)s * n, c->st);
        BatchRequest q;
        q.nsrc = nsrc;
        q.eta = probe;
        q.psi = (const ZD*)xi;
        q.k = ks.data();
        q.jsum = j_out + (size_t)part * 4 * V;
        CHK(run_batched(c, q));
        tslov::launch_current_finish(c->g, q.jsum, 1.0 / nsrc, div_out ? div_out + (size_t)part * V : nullptr,
                                     tot_out ? tot_out + (size_t)part * V : nullptr, c->st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return TSLOV_OK;
}

tslov_status tslov_error_estimate(tslov_ctx* c, const void* psi, int k, const tslov_deflation* defl,
                                  double* eps_out) {
    CHK(check_common(c, k, defl));
    if (!psi || !eps_out) return fail(TSLOV_ERR_ARG, "null argument");
    // canonical buffers 0..2 serve the deflated sign; y and z take 3 and 4
    CHK(ensure(c->canon, (size_t)kCanonBufs * 12 * c->g.V * sizeof(ZD)));
    ZD* y = canon_buf(c, 3);
    CHK(sign_dispatch(c, psi, y, k, defl, nullptr, 0, 0));
    return error_of(c, (const ZD*)psi, y, k, defl, eps_out);
}

tslov_status tslov_lanczos_matrix(tslov_ctx* c, const void* psi, int k, void* T_out, tslov_info* info) {
    CHK(check_common(c, k, nullptr));
    if (!psi || !T_out) return fail(TSLOV_ERR_ARG, "null argument");
    CHK(ensure_work(c, 1, k, 0));
    const SrcList L = make_list({0}, {k});
    std::vector<EntryStatus> es;
    const double t0 = now_ms();
    switch (c->precision) {
        case TSLOV_MIXED: CHK((forward<float, float>(c, L, (const ZD*)psi, nullptr, 0, es))); break;
        case TSLOV_FP32_LINKS: CHK((forward<double, float>(c, L, (const ZD*)psi, nullptr, 0, es))); break;
        default: CHK((forward<double, double>(c, L, (const ZD*)psi, nullptr, 0, es)));
    }
    const int ku = es[0].k_used;
    std::vector<ZD> T((size_t)k * k, ZD{0.0, 0.0});
    if (ku > 0) {
        std::vector<ZD> al(ku + 2), ga(ku + 2);
        std::vector<double> be(ku + 2);
        HIPCHK(hipMemcpyAsync(al.data(), c->coef.alpha, (ku + 1) * sizeof(ZD), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(ga.data(), c->coef.gamma, (ku + 1) * sizeof(ZD), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(be.data(), c->coef.beta, (ku + 1) * sizeof(double), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        for (int j = 1; j <= ku; ++j) {
            T[(size_t)(j - 1) * k + (j - 1)] = al[j];
            if (j < ku) {
                T[(size_t)j * k + (j - 1)] = ZD{be[j + 1], 0.0};   // T_{j+1,j} = beta_{j+1}
                T[(size_t)(j - 1) * k + j] = ga[j + 1];            // T_{j,j+1} = gamma_{j+1}
            }
        }
    }
    std::memcpy(T_out, T.data(), T.size() * sizeof(ZD));
    if (ku > 0) {
        std::vector<ZD> al(ku + 1), ga(ku + 1);
        std::vector<double> be(ku + 1, 0.0);
        for (int j = 0; j < ku; ++j) {
            al[j] = T[(size_t)j * k + j];
            if (j > 0) {
                be[j] = T[(size_t)j * k + (j - 1)].re;
                ga[j] = T[(size_t)(j - 1) * k + j];
            }
        }
        es[0].ritz = tslov::ritz_summary(ku, reinterpret_cast<const double*>(al.data()), be.data(),
                                         reinterpret_cast<const double*>(ga.data()));
        es[0].flags = entry_flags(c, es[0], 0, 0);
    }
    const double ms[6] = {now_ms() - t0, 0, 0, 0, 0, now_ms() - t0};
    fill_info(info, es[0], ms);
    if (es[0].breakdown == 2)
        return fail(TSLOV_ERR_BREAKDOWN, "serious Lanczos breakdown at step " + std::to_string(es[0].step));
    return TSLOV_OK;
}

tslov_status tslov_tridiag_sign(tslov_ctx* c, int k, const double* diag, const double* sub, const double* sup,
                                void* c_out, tslov_info* info) {
    if (!c || !diag || !c_out || (k > 1 && (!sub || !sup))) return fail(TSLOV_ERR_ARG, "null argument");
    if (k < 1 || k > kMaxK) return fail(TSLOV_ERR_ARG, "k must be in [1, 1024]");
    const double t0 = now_ms();
    // coefficient layout of the Lanczos process (step j at index j): alpha_j = T_jj,
    // beta_{j+1} = T_{j+1,j}, gamma_{j+1} = T_{j,j+1}
    std::vector<ZD> al((size_t)k + 2, ZD{0.0, 0.0}), ga((size_t)k + 2, ZD{0.0, 0.0});
    std::vector<double> be((size_t)k + 2, 0.0);
    for (int j = 0; j < k; ++j) {
        al[j + 1] = ZD{diag[2 * j], diag[2 * j + 1]};
        if (j + 1 < k) {
            be[j + 2] = sub[j];
            ga[j + 2] = ZD{sup[2 * j], sup[2 * j + 1]};
        }
    }
    for (int j = 0; j < k; ++j)
        if (!std::isfinite(al[j + 1].re) || !std::isfinite(al[j + 1].im) || !std::isfinite(be[j + 1]) ||
            !std::isfinite(ga[j + 1].re) || !std::isfinite(ga[j + 1].im))
            return fail(TSLOV_ERR_ARG, "the tridiagonal matrix contains non-finite values");
    EntryStatus es;
    es.k_used = k;
    es.ritz = tslov::ritz_summary(k, reinterpret_cast<const double*>(al.data() + 1), be.data() + 1,
                                  reinterpret_cast<const double*>(ga.data() + 1));
    CHK(check_ritz(es));
    CHK(ensure_work(c, 1, k, 0));
    HIPCHK(hipMemcpyAsync(c->coef.alpha, al.data(), al.size() * sizeof(ZD), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->coef.gamma, ga.data(), ga.size() * sizeof(ZD), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->coef.beta, be.data(), be.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    const SrcList L = make_list({0}, {k});
    std::vector<int> iters, stag;
    CHK(dense_step(c, L, 0, iters, &stag));
    HIPCHK(hipMemcpyAsync(c_out, c->coef.c + 1, (size_t)k * sizeof(ZD), hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    es.iters = iters[0];
    es.flags = entry_flags(c, es, stag[0], 0);
    const double ms[6] = {0.0, now_ms() - t0, 0.0, 0.0, 0.0, now_ms() - t0};
    fill_info(info, es, ms);
    return TSLOV_OK;
}

tslov_status tslov_ritz_values(int k, const double* diag, const double* sub, const double* sup, double* out,
                               int* sweeps) {
    if (k < 1 || !diag || !out || (k > 1 && (!sub || !sup))) return fail(TSLOV_ERR_ARG, "bad argument");
    std::vector<double> be((size_t)k, 0.0), ga((size_t)2 * k, 0.0);
    for (int j = 1; j < k; ++j) {
        be[j] = sub[j - 1];
        ga[2 * j] = sup[2 * (j - 1)];
        ga[2 * j + 1] = sup[2 * (j - 1) + 1];
    }
    const int sw = tslov::tridiag_eigvals(k, diag, be.data(), ga.data(), out);
    if (sweeps) *sweeps = sw;
    return TSLOV_OK;
}

tslov_status tslov_block_sign_deflated(tslov_ctx* c, int nu, int site, const double* X, const void* x1,
                                       const void* x2, int k, const tslov_deflation* defl, void* y1_out,
                                       void* y2_out, tslov_info* info) {
    CHK(check_common(c, k, defl));
    if (!x2 || !y1_out || !y2_out) return fail(TSLOV_ERR_ARG, "null argument");
    if (y1_out == y2_out || y1_out == x1 || y1_out == x2 || y2_out == x1 || y2_out == x2)
        return fail(TSLOV_ERR_ARG, "outputs must not overlap each other or the inputs");
    tslov::BlockTangent t;
    CHK(block_args(c, nu, site, X, t));
    DeflSet d;
    CHK(prepare_defl(c, defl, d));
    const double t0 = now_ms();
    EntryStatus es;
    CHK(block_any(c, t, d, d.l ? defl->lambda : nullptr, (const ZD*)x1, (const ZD*)x2, k, (ZD*)y1_out,
                  (ZD*)y2_out, es));
    const double ms[6] = {0.0, 0.0, 0.0, 0.0, 0.0, now_ms() - t0};
    fill_info(info, es, ms);
    return TSLOV_OK;
}

tslov_status tslov_block_sign(tslov_ctx* c, int nu, int site, const double* X, const void* x1, const void* x2,
                              int k, void* y1_out, void* y2_out, tslov_info* info) {
    return tslov_block_sign_deflated(c, nu, site, X, x1, x2, k, nullptr, y1_out, y2_out, info);
}

tslov_status tslov_block_error_estimate_deflated(tslov_ctx* c, int nu, int site, const double* X, const void* psi,
                                                 int k, const tslov_deflation* defl, double* eps_out) {
    CHK(check_common(c, k, defl));
    if (!psi || !eps_out) return fail(TSLOV_ERR_ARG, "null argument");
    tslov::BlockTangent t;
    CHK(block_args(c, nu, site, X, t));
    DeflSet d;
    CHK(prepare_defl(c, defl, d));
    return block_eps(c, t, (const ZD*)psi, k, eps_out, nullptr, d, d.l ? defl->lambda : nullptr);
}

tslov_status tslov_block_error_estimate(tslov_ctx* c, int nu, int site, const double* X, const void* psi, int k,
                                        double* eps_out) {
    return tslov_block_error_estimate_deflated(c, nu, site, X, psi, k, nullptr, eps_out);
}

tslov_status tslov_tune_k(tslov_ctx* c, int ncand, const int* k_outer, const int* k_inner, double trial_target,
                          const tslov_deflation* defl, const tslov_link_direction* dir, int nrand, const void* rand,
                          double* eps_out, double* ms_out, int* chosen, double* cross_out) {
    CHK(check_common(c, 1, defl));
    if (ncand < 1 || !k_outer || !eps_out || !ms_out || !chosen) return fail(TSLOV_ERR_ARG, "null argument");
    if (nrand < 0 || (nrand > 0 && (!rand || !cross_out))) return fail(TSLOV_ERR_ARG, "nrand needs rand and cross_out");
    if (!(trial_target >= 0.0)) return fail(TSLOV_ERR_ARG, "trial_target must be >= 0");
    for (int i = 0; i < ncand; ++i) {
        if (k_outer[i] < 1 || k_outer[i] > kMaxK) return fail(TSLOV_ERR_ARG, "every k_outer must be in [1, 1024]");
        const int ki = k_inner ? k_inner[i] : 0;
        if (ki < 0 || ki > kMaxK) return fail(TSLOV_ERR_ARG, "every k_inner must be in [0, 1024]");
        if (dir && ki != 0) return fail(TSLOV_ERR_ARG, "the block-matrix process has no nested step (k_inner = 0)");
    }
    tslov::BlockTangent t{};
    if (dir) CHK(block_args(c, dir->nu, dir->site, dir->X, t));
    const size_t n12 = (size_t)12 * c->g.V;
    CHK(ensure(c->canon, (size_t)kCanonBufs * n12 * sizeof(ZD)));
    CHK(ensure(c->trial, n12 * sizeof(ZD)));
    {
        const std::vector<ZD> ones(n12, ZD{1.0, 0.0});
        HIPCHK(hipMemcpyAsync(c->trial.p, ones.data(), n12 * sizeof(ZD), hipMemcpyHostToDevice, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
    }
    const ZD* phi = c->trial.as<ZD>();
    for (int i = 0; i < ncand; ++i)
        CHK(tune_candidate(c, phi, k_outer[i], k_inner ? k_inner[i] : 0, defl, dir ? &t : nullptr, &eps_out[i],
                           &ms_out[i]));
    // the fastest candidate within the trial target (the first of equal times)
    int best = -1;
    for (int i = 0; i < ncand; ++i)
        if (eps_out[i] <= trial_target && (best < 0 || ms_out[i] < ms_out[best])) best = i;
    *chosen = best;
    if (best >= 0)
        for (int r = 0; r < nrand; ++r) {
            double ms = 0.0;
            CHK(tune_candidate(c, (const ZD*)rand + (size_t)r * n12, k_outer[best], k_inner ? k_inner[best] : 0, defl,
                               dir ? &t : nullptr, &cross_out[r], &ms));
        }
    return TSLOV_OK;
}

tslov_status tslov_set_nested(tslov_ctx* c, int k_inner) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (k_inner < 0 || k_inner > kMaxK) return fail(TSLOV_ERR_ARG, "k_inner must be in [0, 1024]");
    c->nest_m = k_inner;
    return TSLOV_OK;
}

tslov_status tslov_set_diagnostics(tslov_ctx* c, int flags) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (flags & ~TSLOV_DIAG_EPS_A) return fail(TSLOV_ERR_ARG, "unknown diagnostics flag");
    c->diag = flags;
    return TSLOV_OK;
}

tslov_status tslov_dense_sign(tslov_ctx* c, const void* T, int k, const void* E, void* S_out, void* L_out,
                              int* iters) {
    if (!c || !T || !S_out) return fail(TSLOV_ERR_ARG, "null argument");
    if (k < 1 || k > kMaxK) return fail(TSLOV_ERR_ARG, "k must be in [1, 1024]");
    if (E && !L_out) return fail(TSLOV_ERR_ARG, "L_out required when E is given");
    DenseWork w;
    CHK(ensure_dense(c, 1, k, w));
    tslov::launch_dense_load((const ZD*)T, (const ZD*)E, k, w, c->st);
    const SrcList L = make_list({0}, {k});
    std::vector<int> it;
    CHK(newton(c, L, E ? 1 : 0, w, it, 0));
    const size_t bytes = (size_t)k * k * sizeof(ZD);
    HIPCHK(hipMemcpyAsync(S_out, w.X, bytes, hipMemcpyDeviceToDevice, c->st));
    if (E) HIPCHK(hipMemcpyAsync(L_out, w.Y, bytes, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (iters) *iters = it[0];
    return TSLOV_OK;
}

tslov_status tslov_timing_enable(tslov_ctx* c, int every) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (every < 0) return fail(TSLOV_ERR_ARG, "every must be >= 0");
    c->timing = every;
    for (auto& n : c->tcount) n = 0;
    return TSLOV_OK;
}

tslov_status tslov_timing_read(tslov_ctx* c, int which, int* count, double* total_ms) {
    if (!c || which < 0 || which >= kTimingClasses) return fail(TSLOV_ERR_ARG, "bad argument");
    HIPCHK(hipStreamSynchronize(c->st));
    double tot = 0.0;
    int n = 0;
    for (auto& pr : c->ev_used[which]) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
            tot += ms;
            ++n;
        }
        c->ev_free.push_back(pr.first);
        c->ev_free.push_back(pr.second);
    }
    c->ev_used[which].clear();
    if (count) *count = n;
    if (total_ms) *total_ms = tot;
    return TSLOV_OK;
}

tslov_status tslov_set_graphs(tslov_ctx* c, int on) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (on && !c->st) return fail(TSLOV_ERR_ARG, "graph capture needs a context created on a non-null stream");
    HIPCHK(hipStreamSynchronize(c->st));
    c->graphs = on ? 1 : 0;
    if (!on) {
        c->gfwd.reset();
        c->gbwd.reset();
    }
    return TSLOV_OK;
}

tslov_status tslov_set_apply_chunk(tslov_ctx* c, int T) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (T < 0 || (T > 0 && c->g.nt % T != 0)) return fail(TSLOV_ERR_ARG, "T must be 0 or divide the time extent");
    c->tm_T_forced = T;
    return TSLOV_OK;
}

tslov_status tslov_get_apply_chunk(const tslov_ctx* c, int* T) {
    if (!c || !T) return fail(TSLOV_ERR_ARG, "null argument");
    *T = c->tm_T > 0 ? c->tm_T : 0;
    return TSLOV_OK;
}

tslov_status tslov_set_pair_ns(tslov_ctx* c, int ns) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (ns != 0 && ns != 1 && ns != 2 && ns != 4) return fail(TSLOV_ERR_ARG, "ns must be 0, 1, 2 or 4");
    c->pair_ns_forced = ns;
    return TSLOV_OK;
}

tslov_status tslov_set_cg_operator(tslov_ctx* c, int form) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (form < tslov::kCgOpMulti || form > tslov::kCgOpTmarch) return fail(TSLOV_ERR_ARG, "form must be 0, 1, 2 or 3");
    c->cg_op = form;
    return TSLOV_OK;
}

tslov_status tslov_get_pair_ns(const tslov_ctx* c, int* fwd_ns, int* bwd_ns) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    if (fwd_ns) *fwd_ns = c->pair_ns[0];
    if (bwd_ns) *bwd_ns = c->pair_ns[1];
    return TSLOV_OK;
}

double tslov_kernel_bytes(const tslov_ctx* c, int which) {
    if (!c) return 0.0;
    const double z = (double)c->zsize(), zl = (double)c->lsize();
    const double V = (double)c->g.V;
    switch (which) {
        case 0: return V * (6 * 12 * z + 36 * zl);      // read r, s, links; write v, w, a, b
        case 1: return V * (12 * 12 * z + 36 * zl);     // read 9 fields and links; write 3 fields
        case 2: return V * (2 * 12 * z + 36 * zl);      // read in and links; write out
        default: return 0.0;
    }
}

}  // extern "C"
