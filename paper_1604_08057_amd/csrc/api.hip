// C ABI of the tslov library (declared in include/tslov.h): context and
// workspace management, and the host drivers of the TSL forward pass, the
// projected-matrix Newton step and the reverse-mode pass for dS/dU.
#include "tslov.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"

using tslov::Coef;
using tslov::DenseWork;
using tslov::Geom;
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

}  // namespace

struct tslov_ctx {
    Geom g{};
    double kappa = 0.0, mu = 0.0;
    int antiperiodic = 1, precision = TSLOV_FP64;
    hipStream_t st = nullptr;
    int device = 0;
    size_t lds_max = 65536;
    int links_set = 0;
    Buf U64, U32;
    Buf fields;      // psi, eta, r, s, a, b in the working precision
    Buf basisV, basisW, basisA, basisB;   // v_j, w_j, a_j = H v_j, b_j = H^dag w_j
    Buf abarS, sbarS;
    Buf bwork;       // vbar, wbar, rbar ring
    Buf part;        // partial sums (4 arrays)
    Buf coefmem;
    Buf dense, denseInt, denseLog, densePart;
    Buf gpart;
    Buf canon;       // three canonical spinors: projected source, partial result, error estimate
    Buf deflw;       // deflation coefficients, signs and partial sums
    double* host_part = nullptr;  // pinned
    int host_part_n = 0;
    int kcap = 0;
    Coef coef{};
    int status_init[4] = {0, 0, 0, 0};
    int timing = 0;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[kTimingClasses];

    int nblk() const { return tslov::grid_for(g.V); }
    size_t field_elems() const { return (size_t)12 * g.ldv; }
    size_t zsize() const { return precision == TSLOV_MIXED ? sizeof(Z<float>) : sizeof(ZD); }
    size_t field_bytes() const { return field_elems() * zsize(); }
};

namespace {

// ---------------------------------------------------------------- timing
struct TimedLaunch {
    tslov_ctx* c;
    int cls;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(tslov_ctx* ctx, int which) : c(ctx), cls(which) {
        if (!c->timing) return;
        a = take();
        b = take();
        if (a && b) (void)hipEventRecord(a, c->st);
    }
    hipEvent_t take() {
        if (c->ev_free.empty()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            return e;
        }
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    ~TimedLaunch() {
        if (!c->timing || !a || !b) return;
        (void)hipEventRecord(b, c->st);
        c->ev_used[cls].push_back({a, b});
    }
};

tslov_status ensure_coef(tslov_ctx* c, int k) {
    if (c->kcap >= k && c->coefmem.p) return TSLOV_OK;
    const int n = k + 2;
    const size_t bytes = (size_t)n * (7 * sizeof(ZD) + 4 * sizeof(double)) + 16 * sizeof(int) + 16 * sizeof(double);
    CHK(ensure(c->coefmem, bytes));
    char* p = c->coefmem.as<char>();
    auto take = [&](size_t b) {
        char* q = p;
        p += b;
        return q;
    };
    Coef& cf = c->coef;
    cf.alpha = (ZD*)take(n * sizeof(ZD));
    cf.gamma = (ZD*)take(n * sizeof(ZD));
    cf.h = (ZD*)take(n * sizeof(ZD));
    cf.c = (ZD*)take(n * sizeof(ZD));
    cf.abar_T = (ZD*)take(n * sizeof(ZD));
    cf.gbar_T = (ZD*)take(n * sizeof(ZD));
    cf.gbar_tot = (ZD*)take(n * sizeof(ZD));
    cf.beta = (double*)take(n * sizeof(double));
    cf.anorm2 = (double*)take(n * sizeof(double));
    cf.bbar_T = (double*)take(n * sizeof(double));
    cf.bbar_tot = (double*)take(n * sizeof(double));
    cf.misc = (double*)take(16 * sizeof(double));
    cf.status = (int*)take(16 * sizeof(int));
    c->kcap = k;
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

// Partial-sum arrays: [0] forward pair / RB, [1] recurrence / RA, [2] misc, [3] dense.
double* part_array(tslov_ctx* c, int i) { return c->part.as<double>() + (size_t)i * 8 * tslov::np_max(c->g.V); }

tslov_status ensure_part(tslov_ctx* c) {
    return ensure(c->part, (size_t)4 * 8 * tslov::np_max(c->g.V) * sizeof(double));
}

template <typename R>
Z<R>* fld(const Buf& b, const tslov_ctx* c, int i) { return b.as<Z<R>>() + (size_t)i * c->field_elems(); }

template <typename R>
const Z<R>* links(const tslov_ctx* c) {
    if constexpr (sizeof(R) == sizeof(double)) return c->U64.as<Z<R>>();
    else return c->U32.as<Z<R>>();
}

// ---------------------------------------------------------------- forward
// Fields: 0 psi, 1 eta, 2 r, 3 s, 4 a, 5 b.
template <typename R>
tslov_status forward(tslov_ctx* c, const ZD* psi, const ZD* eta, int k, int* k_used, int* breakdown) {
    const Geom& g = c->g;
    const int np_norm = c->nblk(), np_st = tslov::np_stencil(g.V), np_pt = tslov::np_point(g.V);
    CHK(ensure(c->fields, 6 * c->field_elems() * sizeof(Z<R>)));
    CHK(ensure(c->basisV, (size_t)k * c->field_elems() * sizeof(Z<R>)));
    CHK(ensure(c->basisW, (size_t)k * c->field_elems() * sizeof(Z<R>)));
    CHK(ensure(c->basisA, (size_t)k * c->field_elems() * sizeof(Z<R>)));
    CHK(ensure(c->basisB, (size_t)k * c->field_elems() * sizeof(Z<R>)));
    CHK(ensure_part(c));
    CHK(ensure_coef(c, k));
    Z<R>* X = fld<R>(c->fields, c, 0);
    Z<R>* E = fld<R>(c->fields, c, 1);
    Z<R>* Rf = fld<R>(c->fields, c, 2);
    Z<R>* Sf = fld<R>(c->fields, c, 3);
    double* p_pair = part_array(c, 0);
    double* p_rec = part_array(c, 1);
    c->status_init[0] = 0;
    c->status_init[1] = k;
    c->status_init[2] = 0;
    c->status_init[3] = 0;
    HIPCHK(hipMemcpyAsync(c->coef.status, c->status_init, sizeof(c->status_init), hipMemcpyHostToDevice, c->st));
    tslov::launch_spinor_to_soa<R>(psi, X, g, p_rec, c->st);
    if (eta) tslov::launch_spinor_to_soa<R>(eta, E, g, nullptr, c->st);
    const Z<R>* U = links<R>(c);
    for (int j = 1; j <= k; ++j) {
        Z<R>* vj = fld<R>(c->basisV, c, j - 1);
        Z<R>* wj = fld<R>(c->basisW, c, j - 1);
        Z<R>* Af = fld<R>(c->basisA, c, j - 1);
        Z<R>* Bf = fld<R>(c->basisB, c, j - 1);
        {
            TimedLaunch tl(c, 0);
            tslov::launch_fwd_pair<R>(U, g, c->kappa, c->mu, j == 1 ? X : Rf, j == 1 ? X : Sf, p_rec,
                                      j == 1 ? np_norm : np_pt, j == 1, c->coef, j, vj, wj, Af, Bf, eta ? E : nullptr,
                                      p_pair, c->st);
        }
        tslov::launch_recur<R>(g, Af, Bf, vj, wj, j > 1 ? fld<R>(c->basisV, c, j - 2) : nullptr,
                               j > 1 ? fld<R>(c->basisW, c, j - 2) : nullptr, p_pair, np_st, c->coef, j, j == k, Rf,
                               Sf, p_rec, c->st);
    }
    HIPCHK(hipGetLastError());
    int st[4];
    HIPCHK(hipMemcpyAsync(st, c->coef.status, sizeof(st), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    *k_used = st[1];
    *breakdown = st[2];
    if (st[2] == 2)
        return fail(TSLOV_ERR_BREAKDOWN, "serious Lanczos breakdown at step " + std::to_string(st[3]));
    return TSLOV_OK;
}

// ---------------------------------------------------------------- projected-matrix step
tslov_status ensure_dense(tslov_ctx* c, int k, DenseWork& w) {
    const size_t kk = (size_t)k * k;
    CHK(ensure(c->dense, 5 * kk * sizeof(ZD)));
    CHK(ensure(c->denseInt, (size_t)2 * k * sizeof(int)));
    CHK(ensure(c->denseLog, (size_t)k * sizeof(double)));
    const int np = tslov::grid_for((int)kk, 256);
    CHK(ensure(c->densePart, (size_t)(4 * np + 8) * sizeof(double)));
    CHK(ensure_host_part(c, 2 * np + 8));
    ZD* d = c->dense.as<ZD>();
    w.X = d;
    w.Y = d + kk;
    w.Wk = d + 2 * kk;
    w.Xinv = d + 3 * kk;
    w.Zt = d + 4 * kk;
    w.rowperm = c->denseInt.as<int>();
    w.logpiv = c->denseLog.as<double>();
    w.part = c->densePart.as<double>();
    w.npart_max = np;
    return TSLOV_OK;
}

int choose_nb(const tslov_ctx* c, int k) {
    for (int nb : {16, 8, 4, 2, 1})
        if ((size_t)(k * (nb + 1)) * sizeof(ZD) + (size_t)k * sizeof(int) + 2048 <= c->lds_max) return nb;
    return 1;
}

// Newton iteration on X (and Y) until the relative step falls to rounding level.
tslov_status newton(tslov_ctx* c, int k, int grad, DenseWork& w, int* iters_out) {
    const int nb = choose_nb(c, k);
    int scaling = 1, extra = grad ? 1 : 0, it = 0;
    double prev = INFINITY;
    bool done = false;
    for (it = 1; it <= 100 && !done; ++it) {
        const int np = tslov::dense_newton_step(k, grad, scaling, nb, c->lds_max, w, c->st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(c->host_part, w.part, (size_t)2 * np * sizeof(double), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        double dif = 0.0, nrm = 0.0;
        for (int i = 0; i < np; ++i) {
            dif += c->host_part[2 * i];
            nrm += c->host_part[2 * i + 1];
        }
        const double delta = std::sqrt(dif / nrm);
        if (!std::isfinite(delta))
            return fail(TSLOV_ERR_SIGN_UNDEFINED, "projected matrix is singular or its sign is undefined");
        if (delta < 1e-2) scaling = 0;
        // quadratic convergence: once the step is below 1e-8 the new iterate's error
        // is at rounding level; stagnation above that also ends the iteration
        const bool conv = delta <= 1e-8 || (delta < 1e-6 && delta > 0.5 * prev);
        if (conv) {
            if (extra) extra = 0;
            else done = true;
        }
        prev = delta;
    }
    if (iters_out) *iters_out = it - 1;
    if (!done)
        return fail(TSLOV_ERR_SIGN_UNDEFINED,
                    "sign iteration of the projected matrix did not converge (eigenvalue near Re z = 0)");
    return TSLOV_OK;
}

// ---------------------------------------------------------------- backward
// bwork fields: 0 vbar, 1 wbar, 2/3 rbar ring.
template <typename R>
tslov_status backward(tslov_ctx* c, int k, ZD* dU, ZD* dpsi) {
    const Geom& g = c->g;
    const int np_st = tslov::np_stencil(g.V), np_pt = tslov::np_point(g.V);
    CHK(ensure(c->abarS, (size_t)k * c->field_elems() * sizeof(Z<R>)));
    CHK(ensure(c->sbarS, (size_t)k * c->field_elems() * sizeof(Z<R>)));
    CHK(ensure(c->bwork, 4 * c->field_elems() * sizeof(Z<R>)));
    Z<R>* VB = fld<R>(c->bwork, c, 0);
    Z<R>* WB = fld<R>(c->bwork, c, 1);
    Z<R>* X = fld<R>(c->fields, c, 0);
    Z<R>* E = fld<R>(c->fields, c, 1);
    double* p_rb = part_array(c, 0);
    double* p_ra = part_array(c, 1);
    const Z<R>* U = links<R>(c);
    auto V = [&](int j) { return fld<R>(c->basisV, c, j - 1); };   // v_j, 1-based
    auto W = [&](int j) { return fld<R>(c->basisW, c, j - 1); };
    auto A = [&](int j) { return fld<R>(c->basisA, c, j - 1); };
    auto B = [&](int j) { return fld<R>(c->basisB, c, j - 1); };
    auto RB = [&](int j) { return fld<R>(c->bwork, c, 2 + (j & 1)); };
    auto SB = [&](int j) { return fld<R>(c->sbarS, c, j - 1); };
    auto AB = [&](int j) { return fld<R>(c->abarS, c, j - 1); };
    for (int j = k; j >= 1; --j) {
        if (j < k)
            tslov::launch_bwd_ra<R>(g, VB, WB, V(j + 1), W(j + 1), V(j), W(j), j > 1 ? V(j - 1) : nullptr,
                                    j > 1 ? W(j - 1) : nullptr, p_rb, np_st, c->coef, j, RB(j), SB(j), p_ra, c->st);
        TimedLaunch tl(c, 1);
        tslov::launch_bwd_rb<R>(U, g, c->kappa, c->mu, p_ra, np_pt, c->coef, j, k, RB(j), RB(j + 1), SB(j),
                                j < k ? SB(j + 1) : SB(j), V(j), W(j), A(j), B(j), E, VB, WB, AB(j), p_rb, c->st);
    }
    // force contraction over all steps, split in chunks of j for parallelism
    int nchunk = (1 << 18) / (4 * g.V);
    if (nchunk < 1) nchunk = 1;
    if (nchunk > k) nchunk = k;
    if (nchunk > 64) nchunk = 64;
    CHK(ensure(c->gpart, (size_t)nchunk * 36 * g.ldv * sizeof(ZD)));
    tslov::launch_force<R>(g, c->kappa, c->mu, AB(1), SB(1), V(1), W(1), c->field_elems(), c->coef.status, nchunk,
                           c->gpart.as<ZD>(), c->st);
    tslov::launch_force_reduce(g, c->gpart.as<ZD>(), nchunk, c->antiperiodic, dU, c->st);
    if (dpsi) tslov::launch_source_grad<R>(g, VB, WB, X, c->coef, part_array(c, 2), dpsi, c->st);
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

ZD* canon_buf(tslov_ctx* c, int i) { return c->canon.as<ZD>() + (size_t)i * 12 * c->g.V; }

// out = [psi +] g5^{overlap} sgn(H) psi by TSL, with optional deflation.
template <typename R>
tslov_status sign_impl(tslov_ctx* c, const void* psi_in, void* out, int k, const tslov_deflation* defl,
                       tslov_info* info, int overlap) {
    const double t0 = now_ms();
    DeflSet d;
    CHK(prepare_defl(c, defl, d));
    const ZD* psi = (const ZD*)psi_in;
    const ZD* src = psi;
    if (d.l) {
        CHK(ensure(c->canon, (size_t)3 * 12 * c->g.V * sizeof(ZD)));
        tslov::launch_defl_coeffs(d.L, psi, c->g.V, d.l, d.part, d.c, c->st);
        tslov::launch_defl_project(d.R, psi, d.c, c->g.V, d.l, canon_buf(c, 0), c->st);
        src = canon_buf(c, 0);
    }
    int k_used = 0, bd = 0;
    CHK(forward<R>(c, src, nullptr, k, &k_used, &bd));
    const double t1 = now_ms();
    int iters = 0;
    if (k_used > 0) {
        DenseWork w;
        CHK(ensure_dense(c, k_used, w));
        tslov::launch_dense_build(c->coef, k_used, 0, w, c->st);
        CHK(newton(c, k_used, 0, w, &iters));
        tslov::launch_dense_extract(c->coef, k_used, 0, w, c->st);
    }
    const double t2 = now_ms();
    if (d.l) {
        ZD* yp = nullptr;
        if (k_used > 0) {
            yp = canon_buf(c, 1);
            tslov::launch_assemble<R>(c->g, c->basisV.as<Z<R>>(), c->field_elems(), c->coef, nullptr, 0, yp, c->st);
        }
        tslov::launch_defl_finish(d.R, d.c, d.sgn, yp, psi, c->g.V, d.l, overlap, (ZD*)out, c->st);
    } else if (k_used > 0) {
        tslov::launch_assemble<R>(c->g, c->basisV.as<Z<R>>(), c->field_elems(), c->coef, psi, overlap, (ZD*)out,
                                  c->st);
    } else {
        tslov::launch_defl_finish(nullptr, nullptr, nullptr, nullptr, psi, c->g.V, 0, overlap, (ZD*)out, c->st);
    }
    HIPCHK(hipGetLastError());
    double nx = 0.0;
    HIPCHK(hipMemcpyAsync(&nx, c->coef.misc, sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    const double t3 = now_ms();
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->k_used = k_used;
        info->breakdown = bd;
        info->newton_iters = iters;
        info->norm_x = nx;
        info->ms[0] = t1 - t0;
        info->ms[1] = t2 - t1;
        info->ms[2] = t3 - t2;
        info->ms[5] = t3 - t0;
    }
    return TSLOV_OK;
}

template <typename R>
tslov_status grad_impl(tslov_ctx* c, const void* eta, const void* psi, int k, double* S_out, void* dU, void* dpsi,
                       tslov_info* info) {
    const double t0 = now_ms();
    int k_used = 0, bd = 0;
    CHK(forward<R>(c, (const ZD*)psi, (const ZD*)eta, k, &k_used, &bd));
    const double t1 = now_ms();
    if (k_used == 0) {   // zero source: S = 0 and every derivative vanishes
        HIPCHK(hipMemsetAsync(dU, 0, (size_t)36 * c->g.V * sizeof(ZD), c->st));
        if (dpsi) HIPCHK(hipMemsetAsync(dpsi, 0, (size_t)12 * c->g.V * sizeof(ZD), c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        if (S_out) *S_out = 0.0;
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->breakdown = bd;
        }
        return TSLOV_OK;
    }
    DenseWork w;
    CHK(ensure_dense(c, k_used, w));
    tslov::launch_dense_build(c->coef, k_used, 1, w, c->st);
    int iters = 0;
    CHK(newton(c, k_used, 1, w, &iters));
    tslov::launch_dense_extract(c->coef, k_used, 1, w, c->st);
    const double t2 = now_ms();
    CHK(backward<R>(c, k_used, (ZD*)dU, (ZD*)dpsi));
    double misc[2] = {0.0, 0.0};
    HIPCHK(hipMemcpyAsync(misc, c->coef.misc, sizeof(misc), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    const double t3 = now_ms();
    if (S_out) *S_out = misc[1];
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->k_used = k_used;
        info->breakdown = bd;
        info->newton_iters = iters;
        info->norm_x = misc[0];
        info->ms[0] = t1 - t0;
        info->ms[1] = t2 - t1;
        info->ms[3] = t3 - t2;
        info->ms[5] = t3 - t0;
    }
    return TSLOV_OK;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

const char* tslov_last_error(void) { return g_err.c_str(); }

tslov_status tslov_create(const tslov_lattice_desc* d, void* stream, tslov_ctx** out) {
    if (!d || !out) return fail(TSLOV_ERR_ARG, "null argument");
    *out = nullptr;
    for (int i = 0; i < 4; ++i)
        if (d->dims[i] < 2) return fail(TSLOV_ERR_ARG, "every lattice extent must be >= 2");
    if (d->precision != TSLOV_FP64 && d->precision != TSLOV_MIXED) return fail(TSLOV_ERR_ARG, "unknown precision");
    if (2.0 * d->mass + 8.0 == 0.0) return fail(TSLOV_ERR_ARG, "2*mass + 8 must be non-zero");
    const long long V = (long long)d->dims[0] * d->dims[1] * d->dims[2] * d->dims[3];
    if (V > (1LL << 26)) return fail(TSLOV_ERR_ARG, "lattice volume too large");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    tslov_ctx* c = new tslov_ctx();
    c->device = dev;
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
    if (s == TSLOV_OK && c->precision == TSLOV_MIXED) s = ensure(c->U32, (size_t)36 * c->g.ldv * sizeof(Z<float>));
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
    for (Buf* b : {&c->U64, &c->U32, &c->fields, &c->basisV, &c->basisW, &c->basisA, &c->basisB, &c->abarS, &c->sbarS,
                   &c->bwork, &c->part, &c->canon, &c->deflw,
                   &c->coefmem, &c->dense, &c->denseInt, &c->denseLog, &c->densePart, &c->gpart})
        release(*b);
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
    tslov::launch_links_to_soa((const ZD*)U, c->U64.as<ZD>(), c->precision == TSLOV_MIXED ? c->U32.as<Z<float>>() : nullptr,
                               c->g, c->antiperiodic, c->st);
    HIPCHK(hipGetLastError());
    c->links_set = 1;
    return TSLOV_OK;
}

static tslov_status apply_op(tslov_ctx* c, const void* in, void* out, double mu, int g5in, int g5out) {
    if (!c || !in || !out) return fail(TSLOV_ERR_ARG, "null argument");
    if (!c->links_set) return fail(TSLOV_ERR_ARG, "links not set (call tslov_set_links first)");
    if (in == out) return fail(TSLOV_ERR_ARG, "in and out must not overlap");
    CHK(ensure(c->fields, 6 * c->field_bytes()));
    if (c->precision == TSLOV_MIXED) {
        Z<float>* a = fld<float>(c->fields, c, 0);
        Z<float>* b = fld<float>(c->fields, c, 1);
        tslov::launch_spinor_to_soa<float>((const ZD*)in, a, c->g, nullptr, c->st);
        {
            TimedLaunch tl(c, 2);
            tslov::launch_apply<float>(c->U32.as<Z<float>>(), a, b, c->g, c->kappa, mu, g5in, g5out, c->st);
        }
        tslov::launch_spinor_from_soa<float>(b, (ZD*)out, c->g, c->st);
    } else {
        ZD* a = fld<double>(c->fields, c, 0);
        ZD* b = fld<double>(c->fields, c, 1);
        tslov::launch_spinor_to_soa<double>((const ZD*)in, a, c->g, nullptr, c->st);
        {
            TimedLaunch tl(c, 2);
            tslov::launch_apply<double>(c->U64.as<ZD>(), a, b, c->g, c->kappa, mu, g5in, g5out, c->st);
        }
        tslov::launch_spinor_from_soa<double>(b, (ZD*)out, c->g, c->st);
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

tslov_status tslov_sign(tslov_ctx* c, const void* psi, void* out, int k, const tslov_deflation* defl,
                        tslov_info* info) {
    CHK(check_common(c, k, defl));
    if (!psi || !out) return fail(TSLOV_ERR_ARG, "null argument");
    if (psi == out) return fail(TSLOV_ERR_ARG, "psi and out must not overlap");
    return c->precision == TSLOV_MIXED ? sign_impl<float>(c, psi, out, k, defl, info, 0)
                                       : sign_impl<double>(c, psi, out, k, defl, info, 0);
}

tslov_status tslov_overlap(tslov_ctx* c, const void* psi, void* out, int k, const tslov_deflation* defl,
                           tslov_info* info) {
    CHK(check_common(c, k, defl));
    if (!psi || !out) return fail(TSLOV_ERR_ARG, "null argument");
    if (psi == out) return fail(TSLOV_ERR_ARG, "psi and out must not overlap");
    return c->precision == TSLOV_MIXED ? sign_impl<float>(c, psi, out, k, defl, info, 1)
                                       : sign_impl<double>(c, psi, out, k, defl, info, 1);
}

tslov_status tslov_sign_grad(tslov_ctx* c, const void* eta, const void* psi, int k, const tslov_deflation* defl,
                             int recompute_stride, double* S_out, void* dU_out, void* dpsi_out, tslov_info* info) {
    CHK(check_common(c, k, defl));
    if (!eta || !psi || !dU_out) return fail(TSLOV_ERR_ARG, "null argument");
    if (defl && defl->l != 0)
        return fail(TSLOV_ERR_ARG, "the derivative with deflation (eigenpair motion) is not supported; pass NULL");
    if (recompute_stride != 0) return fail(TSLOV_ERR_ARG, "recompute_stride must be 0 (all vectors stored)");
    return c->precision == TSLOV_MIXED ? grad_impl<float>(c, eta, psi, k, S_out, dU_out, dpsi_out, info)
                                       : grad_impl<double>(c, eta, psi, k, S_out, dU_out, dpsi_out, info);
}

tslov_status tslov_error_estimate(tslov_ctx* c, const void* psi, int k, const tslov_deflation* defl,
                                  double* eps_out) {
    CHK(check_common(c, k, defl));
    if (!psi || !eps_out) return fail(TSLOV_ERR_ARG, "null argument");
    const size_t n = (size_t)12 * c->g.V;
    // canonical buffers 0..2 serve the deflated sign; y and z take 3 and 4
    CHK(ensure(c->canon, (size_t)5 * n * sizeof(ZD)));
    CHK(ensure_part(c));
    ZD* y = canon_buf(c, 3);
    ZD* z = canon_buf(c, 4);
    tslov_status s = c->precision == TSLOV_MIXED ? sign_impl<float>(c, psi, y, k, defl, nullptr, 0)
                                                 : sign_impl<double>(c, psi, y, k, defl, nullptr, 0);
    if (s == TSLOV_OK)
        s = c->precision == TSLOV_MIXED ? sign_impl<float>(c, y, z, k, defl, nullptr, 0)
                                        : sign_impl<double>(c, y, z, k, defl, nullptr, 0);
    if (s != TSLOV_OK) return s;
    CHK(ensure_host_part(c, 2048));
    double* part = part_array(c, 2);
    const int nb = tslov::launch_diff_norm(z, (const ZD*)psi, n, part, c->st);
    HIPCHK(hipMemcpyAsync(c->host_part, part, (size_t)2 * nb * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    double dif = 0.0, nrm = 0.0;
    for (int i = 0; i < nb; ++i) {
        dif += c->host_part[2 * i];
        nrm += c->host_part[2 * i + 1];
    }
    // sgn(0) = 0 is exact: a zero source has no error
    *eps_out = nrm > 0.0 ? std::sqrt(dif / nrm) / 2.0 : 0.0;
    return TSLOV_OK;
}

tslov_status tslov_dense_sign(tslov_ctx* c, const void* T, int k, const void* E, void* S_out, void* L_out,
                              int* iters) {
    if (!c || !T || !S_out) return fail(TSLOV_ERR_ARG, "null argument");
    if (k < 1 || k > kMaxK) return fail(TSLOV_ERR_ARG, "k must be in [1, 1024]");
    if (E && !L_out) return fail(TSLOV_ERR_ARG, "L_out required when E is given");
    DenseWork w;
    CHK(ensure_dense(c, k, w));
    tslov::launch_dense_load((const ZD*)T, (const ZD*)E, k, w, c->st);
    CHK(newton(c, k, E ? 1 : 0, w, iters));
    const size_t bytes = (size_t)k * k * sizeof(ZD);
    HIPCHK(hipMemcpyAsync(S_out, w.X, bytes, hipMemcpyDeviceToDevice, c->st));
    if (E) HIPCHK(hipMemcpyAsync(L_out, w.Y, bytes, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return TSLOV_OK;
}

tslov_status tslov_timing_enable(tslov_ctx* c, int enable) {
    if (!c) return fail(TSLOV_ERR_ARG, "null context");
    c->timing = enable ? 1 : 0;
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

double tslov_kernel_bytes(const tslov_ctx* c, int which) {
    if (!c) return 0.0;
    const double z = (double)c->zsize();
    const double V = (double)c->g.V;
    switch (which) {
        case 0: return V * (6 * 12 + 36) * z;           // read r, s, links; write v, w, a, b
        case 1: return V * (12 * 12 + 36) * z;          // read 9 fields and links; write 3 fields
        case 2: return V * (2 * 12 + 36) * z;           // read in and links; write out
        default: return 0.0;
    }
}

}  // extern "C"
