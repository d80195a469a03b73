/*
 * tslov -- two-sided Lanczos sign function of the Wilson-Dirac operator at
 * finite chemical potential and its derivative with respect to the gauge links,
 * on one AMD MI355X (gfx950).
 *
 * Paper: M. Puhr and P. Buividovich, "A numerical method to compute derivatives
 * of functions of large complex matrices and its application to the overlap
 * Dirac operator at finite chemical potential" (arXiv:1604.08057).
 *
 * Canonical layouts (all device pointers unless stated otherwise):
 *   site       s = x + Nx*(y + Ny*(z + Nz*t))           dims = {Nx, Ny, Nz, Nt}
 *   links      U[mu][s][a][b]     complex128, 4*V*9      mu = x, y, z, t; U_mu(s) leaves s
 *   spinors    psi[s][spin][c]    complex128, V*12
 *   complex128 = two doubles (re, im), C99 "double complex" / torch.complex128.
 * Dirac matrices: chiral basis g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]],
 * g_5 = g_1 g_2 g_3 g_4 = diag(1, 1, -1, -1).
 *
 * Ownership: the caller allocates every input and output buffer; the library
 * never frees nor retains them after a call returns.  The library owns its
 * workspace (device memory allocated on demand and kept until tslov_destroy).
 * All device work is enqueued on the stream given to tslov_create.
 *
 * Errors: every call returns a tslov_status; tslov_last_error() gives a
 * human-readable message for the calling thread.  Argument errors are detected
 * before any work is enqueued.  HIP errors surface on the failing call.
 */
#ifndef TSLOV_H
#define TSLOV_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tslov_status {
    TSLOV_OK = 0,
    TSLOV_ERR_ARG = 1,            /* invalid argument; nothing was enqueued            */
    TSLOV_ERR_HIP = 2,            /* a HIP runtime call or kernel launch failed        */
    TSLOV_ERR_OOM = 3,            /* workspace allocation failed                       */
    TSLOV_ERR_BREAKDOWN = 4,      /* serious Lanczos breakdown: s^H r = 0, r != 0      */
    TSLOV_ERR_SIGN_UNDEFINED = 5, /* sign of the projected matrix undefined (Re = 0)   */
    TSLOV_ERR_NOT_CONVERGED = 6   /* an iterative inner step did not converge          */
} tslov_status;

typedef enum tslov_precision {
    TSLOV_FP64 = 0,       /* links, Krylov vectors and stencil in float64                 */
    TSLOV_MIXED = 1,      /* links, Krylov vectors and stencil in float32 with float32
                             accumulation; inner products, Lanczos coefficients, the
                             projected-matrix sign / Frechet step and the output
                             accumulation in float64.  The rounding of every step is
                             amplified by the non-Hermitian recursion: the link
                             derivative is not accurate (see tslov_sign_grad)       */
    TSLOV_FP32_LINKS = 2  /* links stored and read in float32 (widened to float64 as they
                             are loaded); Krylov vectors, stencil arithmetic and every
                             accumulation in float64.  The float32 rounding then acts as
                             one fixed perturbation of the operator instead of fresh
                             noise at every step                                     */
} tslov_precision;

/* Lattice and operator description (App. A, eq. WD_op / WD_G). */
typedef struct tslov_lattice_desc {
    int dims[4];         /* Nx, Ny, Nz, Nt (each >= 2)                                   */
    double mass;         /* signed Wilson mass m; hopping parameter kappa = 1/(2m + 8)   */
    double mu;           /* quark chemical potential: e^{+mu} on forward temporal hops   */
    int antiperiodic_t;  /* 1: antiperiodic in t (factor -1 across t = Nt-1 -> 0)        */
    int precision;       /* tslov_precision                                              */
} tslov_lattice_desc;

/* Bits of tslov_info.flags. */
typedef enum tslov_flag {
    TSLOV_FLAG_SIGN_STAGNATED = 1,    /* the Newton iteration for sgn(T_k) stopped on stagnation with
                                         a last relative step between 1e-8 and 1e-6 (sgn(T_k) is then
                                         accurate to about that step only)                          */
    TSLOV_FLAG_GRAD_FP32_VECTORS = 2, /* a derivative from TSLOV_MIXED: float32 rounding at every
                                         Lanczos step is amplified by the non-Hermitian recursion, so
                                         dU_out and dpsi_out carry errors far above float32 rounding
                                         (measured 0.1 relative and more); use TSLOV_FP32_LINKS or
                                         TSLOV_FP64 where the derivative matters                    */
    TSLOV_FLAG_RITZ_UNSETTLED = 4     /* the eigenvalue iteration for the Ritz values did not settle
                                         for every eigenvalue: min_abs_re_ritz is approximate        */
} tslov_flag;

/* Per-call diagnostics (host struct, valid after the call returns). */
typedef struct tslov_info {
    int k_used;          /* Krylov size reached (< k after a lucky breakdown)           */
    int breakdown;       /* 0 none, 1 lucky (invariant Krylov space), 2 serious           */
    int newton_iters;    /* iterations of the projected-matrix sign step                 */
    int cg_iters;        /* iterations of the shifted solves of a deflated derivative (else 0) */
    int flags;           /* tslov_flag bits                                              */
    int reserved;
    double norm_x;       /* |psi| (of the projected source when deflating)              */
    double min_abs_re_ritz; /* min |Re theta| over the eigenvalues theta of T_{k_used} (the Ritz
                             values whose signs the approximation interpolates), from a host
                             eigenvalue solve of the tridiagonal matrix; NaN if k_used = 0.
                             A value <= 1e-12 norm_T makes the call fail with ERR_SIGN_UNDEFINED
                             (the sign is undefined on Re z = 0, Sec. 2 after eq. spectral_form) */
    double norm_T;       /* infinity norm of T_{k_used} (NaN if k_used = 0)              */
    double biorth_err;   /* |w_1^H v_k| + |w_k^H v_1| with k = k_used and the normalisation
                            w_j^H v_j = 1 (0 for k_used < 2): the entries of W^H V - I farthest
                            from the diagonal, the loss of biorthogonality that the plain
                            recursion accumulates                                         */
    double eps_A;        /* error estimate of Sec. 4.1 eq. error_est for this output; NaN unless
                            requested with tslov_set_diagnostics (single-source calls)     */
    double ms[6];        /* phase times in ms: forward, dense, output, backward,
                            extra (deflation solves, error estimate), total               */
} tslov_info;

typedef struct tslov_ctx tslov_ctx;

/* Create a context on the current HIP device.  `stream` is a hipStream_t (may be
 * NULL for the default stream).  Fails with ERR_ARG for dims < 2 or unknown
 * precision, ERR_HIP if no device is usable. */
tslov_status tslov_create(const tslov_lattice_desc* desc, void* stream, tslov_ctx** out);
void tslov_destroy(tslov_ctx* ctx);
const char* tslov_last_error(void);

/* Copy the gauge field (canonical complex128 [4][V][3][3], device) into the
 * library's structure-of-arrays layout; the antiperiodic sign is folded into
 * the temporal links on the last time slice.  No caller pointer is kept.
 * ERR_ARG (and no links set) if an element is not finite.  Synchronises the
 * stream once (for that check). */
tslov_status tslov_set_links(tslov_ctx* ctx, const void* U);

/* out = D_w(mu) in (dagger = 0) or D_w(mu)^dagger in = g5 D_w(-mu) g5 in
 * (dagger = 1), eq. WD_op.  `in` and `out` are canonical spinors and must not
 * overlap.  Runs in the context precision. */
tslov_status tslov_apply_dw(tslov_ctx* ctx, const void* in, void* out, int dagger);

/* out = H(mu) in = g5 D_w(mu) in (dagger = 0) or H(mu)^dagger in = H(-mu) in (dagger = 1),
 * Sec. 1 (definition after eq. overlap). */
tslov_status tslov_apply_h(tslov_ctx* ctx, const void* in, void* out, int dagger);

/* tslov_apply_h without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operator, same arguments and same result bits as
 * tslov_apply_h, with its two staging fields in a static device array of 32 MiB
 * that each device holds for the life of the process, instead of the context's
 * workspace.  The lattice must fit it: 2 * 12 * V complex values of the context
 * precision (float64 / float32-link contexts: V <= 87381, e.g. up to 16^4; float32:
 * twice that), else ERR_ARG.  It never times launches and never picks the
 * marching chunk length by timing (it uses the context's pick if one was made,
 * else the built-in choice).  Every call on a device shares that device's array:
 * calls that overlap on one device (other streams, other contexts, other threads)
 * race on it and must be serialised by the caller. */
tslov_status tslov_apply_h_noalloc(tslov_ctx* ctx, const void* in, void* out, int dagger);

/* Optional deflation by known eigenpairs of H (Sec. 3: the standard projection
 * for a diagonalisable matrix, eq. final_res without the mixing term):
 *   c_i = L_i^H psi,  psi_p = psi - sum_i c_i R_i,
 *   sgn(H) psi = TSL(psi_p) + sum_i sgn(Re lambda_i) c_i R_i.
 * R, L: l canonical spinors each, contiguous ([l][V][4][3] complex128, device),
 * right and left eigenvectors of H with L_i^H R_j = delta_ij (caller's
 * normalisation; not checked); lambda: host array of 2*l doubles (re, im);
 * 0 <= l <= 256.  An eigenvalue with |Re| <= 1e-12 max|lambda| gives
 * ERR_SIGN_UNDEFINED.  The caller keeps ownership. */
typedef struct tslov_deflation {
    int l;
    const void* R;
    const void* L;
    const double* lambda;
} tslov_deflation;

/* Two-sided Lanczos approximation out = |psi| V_k sgn(T_k) e_1 ~ sgn(H(mu)) psi
 * (Sec. 2: Krylov spaces of H and H^dagger from the same source; v_1 = w_1 = psi/|psi|),
 * k >= 1 basis vectors (k <= 1024).  A lucky breakdown returns OK with
 * info->k_used < k and the exact result on the invariant space; a serious
 * breakdown returns ERR_BREAKDOWN (out undefined); a zero (projected) source
 * gives k_used = 0; a source with a non-finite element gives ERR_ARG.  defl may be NULL.  info may be NULL. */
tslov_status tslov_sign(tslov_ctx* ctx, const void* psi, void* out, int k,
                        const tslov_deflation* defl, tslov_info* info);

/* out = D_ov psi = psi + g5 sgn(H(mu)) psi with lattice spacing a = 1 (eq. overlap),
 * sgn by two-sided Lanczos as in tslov_sign. */
tslov_status tslov_overlap(tslov_ctx* ctx, const void* psi, void* out, int k,
                           const tslov_deflation* defl, tslov_info* info);

/* S = Re <eta | TSL_k(H(U), psi)> and its exact derivative with respect to every
 * link (eq. derivative_def taken through the k-step approximation, with the
 * Frechet derivative of sgn on T_k from Theorem 1):
 *   dU_out[mu][s] = dS/dRe U_mu(s) + i dS/dIm U_mu(s)  (canonical complex128, device),
 *   so dS = Re tr(dU_out^H dU);  the U(1) link-phase derivative is -Im tr(dU_out^H U).
 * dpsi_out (nullable, canonical spinor) receives dS/dRe psi + i dS/dIm psi.
 * S_out is a host pointer.  For D_ov the caller passes g5 eta and adds Re <eta|psi>.
 * recompute_stride = 0 stores every Krylov vector (6*k*12*V complex values of
 * workspace: v_j, w_j, H v_j, H^dag w_j and two reverse-pass fields per step).
 * recompute_stride = m > 0 with m + 2 < k holds m + 2 steps instead, plus four
 * fields per m steps (the Lanczos state at every m-th step): the reverse pass
 * runs in segments of m steps from the top, and each segment first regenerates
 * its vectors by repeating its forward steps with the recorded coefficients, one
 * more stencil pair per step in all.  S is that of recompute_stride = 0 exactly
 * (the forward pass is the same); the regenerated vectors, and with them dU_out
 * and dpsi_out, agree with the stored ones to rounding (measured about 1e-15
 * relative).  ERR_ARG for a negative stride.
 * With defl (l > 0) S is that of the deflated sign (see tslov_deflation) and the
 * derivative includes the motion of the deflated eigenpairs with U (Sec. 3, App. E):
 * for simple eigenvalues dPi_i = Z_i dH Pi_i + Pi_i dH Z_i, Pi_i = R_i L_i^H,
 * Z_i = (lambda_i - H)^{-1}(1 - Pi_i); the 2l systems for Z_i psi and Z_i^H a_i
 * (a_i = s_i eta - dS/dpsi_p) are solved on the device by conjugate gradients on
 * the normal equations to relative residual 1e-11 (ERR_NOT_CONVERGED after 1e5
 * iterations; info->cg_iters = iterations used).  R, L must be accurate
 * eigenvectors of H(U) for the links set (the formula assumes exact eigenpairs);
 * eigenvalues must be distinct.
 * y_out (nullable, canonical spinor) receives the approximation of sgn(H) psi itself
 * (as tslov_sign computes it), formed inside the same call from the same Krylov basis.
 * In TSLOV_MIXED the derivative outputs carry info->flags TSLOV_FLAG_GRAD_FP32_VECTORS. */
tslov_status tslov_sign_grad(tslov_ctx* ctx, const void* eta, const void* psi, int k,
                             const tslov_deflation* defl, int recompute_stride,
                             double* S_out, void* dU_out, void* dpsi_out, void* y_out, tslov_info* info);

/* The same for the overlap operator (eq. overlap, a = 1):
 *   S = Re <eta | D_ov | psi> = Re <eta|psi> + Re <g5 eta | TSL_k(H(U), psi)>,
 * with dU_out = dS/dRe U + i dS/dIm U as in tslov_sign_grad, dpsi_out (nullable)
 * = dS/dpsi = eta + the source gradient of the sign part, and dov_out (nullable)
 * = D_ov psi = psi + g5 TSL_k(H, psi).  Deflation, recompute_stride and info as in
 * tslov_sign_grad (whose derivative with respect to eta is the output y). */
tslov_status tslov_overlap_grad(tslov_ctx* ctx, const void* eta, const void* psi, int k,
                                const tslov_deflation* defl, int recompute_stride,
                                double* S_out, void* dU_out, void* dpsi_out, void* dov_out, tslov_info* info);

/* Batched derivative (many noise sources, uneven Krylov sizes): for s < nsrc,
 *   S_out[s] = Re <eta_s | TSL_{k[s]}(H(U), psi_s)>,  dU_out[s] = dS_s/dRe U + i dS_s/dIm U,
 * each exactly as tslov_sign_grad computes it for that source alone.
 * eta, psi: nsrc canonical spinors, contiguous ([nsrc][V][4][3] complex128, device);
 * k: host array of nsrc Krylov sizes in [1, 1024]; S_out: host array of nsrc
 * doubles (nullable); dU_out: [nsrc][4][V][3][3] complex128 (device); dpsi_out:
 * [nsrc][V][4][3] (nullable); y_out: [nsrc][V][4][3] (nullable) receives each
 * source's sgn(H) psi_s; infos: host array of nsrc (nullable).
 * The library runs the sources in lockstep groups (one launch per Lanczos step
 * serves every active source of the group; a source leaves the group after its
 * own k[s] steps or a lucky breakdown), sized to the free device memory.  A
 * serious breakdown of some sources returns ERR_BREAKDOWN after every other
 * source has been computed (their outputs are valid; the broken ones' are not;
 * infos[s].breakdown = 2 names them). */
tslov_status tslov_sign_grad_batched(tslov_ctx* ctx, int nsrc, const void* eta, const void* psi, const int* k,
                                     double* S_out, void* dU_out, void* dpsi_out, void* y_out,
                                     tslov_info* infos);

/* The batched derivative with deflation: for s < nsrc exactly what tslov_sign_grad
 * computes with defl for that source alone (the same bits), S_s = Re <eta_s | the
 * deflated sign of psi_s>, the derivative including the eigenpairs' motion.  The TSL
 * parts run as one batch (as tslov_sign_grad_batched); the 2l shifted systems of
 * every source run as one batched conjugate-gradient solve of 2l nsrc systems
 * (infos[s].cg_iters = its iterations).  Arguments as tslov_sign_grad_batched, defl as
 * tslov_sign_grad; defl = NULL or l = 0 is tslov_sign_grad_batched.  Workspace: three
 * canonical spinors and 10 l float64 SoA fields per source beyond the batch's. */
tslov_status tslov_sign_grad_batched_deflated(tslov_ctx* ctx, int nsrc, const void* eta, const void* psi,
                                              const int* k, const tslov_deflation* defl, double* S_out,
                                              void* dU_out, void* dpsi_out, void* y_out, tslov_info* infos);

/* Stochastic estimator of the link-current trace (Sec. 4, the U(1) vector current
 * test, eq. lat_vec_cur without the inverse Dirac operator): with Z2 noise xi_s,
 *   j(x, nu) = (1/nsrc) sum_s dS_s/dTheta_{x,nu},  S_s = Re <g5 xi_s | sgn(H) | xi_s>,
 * the derivative with respect to the U(1) phase of U_nu(x) -> e^{i Theta} U_nu(x),
 * i.e. -Im tr(G_s^H U_nu(x)) with G_s the link gradient of tslov_sign_grad.  Since
 * D_ov = 1 + g5 sgn(H), this estimates Re Tr(dD_ov/dTheta_{x,nu}).
 * xi: [nsrc][V][4][3] complex128 (device); k: host array of nsrc sizes;
 * j_out: device double [4][V] (direction-major); div_out, tot_out: device double
 * [V] (nullable) receive the divergence sum_nu [j(x, nu) - j(x - nu, nu)] and the
 * total current sum_nu [j(x, nu) + j(x - nu, nu)] (eq. divergence_def and the sum
 * with the sign flipped).  ward_out (host, nullable): the per-sample Ward
 * identity of the local U(1) symmetry, max over sources and sites of
 * |sum_nu [g_s(x,nu) - g_s(x-nu,nu)] - (-Im eta_s^H y_s + Im dpsi_s^H xi_s)(x)|
 * divided by max |g_s(x, nu)|, with eta_s = g5 xi_s, y_s = TSL(xi_s) and dpsi_s
 * the source gradient; it is zero up to rounding for the exact derivative.
 * Requesting it costs one extra assembly and source gradient per source. */
tslov_status tslov_current_estimate(tslov_ctx* ctx, int nsrc, const void* xi, const int* k, double* j_out,
                                    double* div_out, double* tot_out, double* ward_out, tslov_info* infos);

/* The same estimator with the deflated sign (Sec. 4.3 with Sec. 3): every term the U(1)
 * projection of the deflated link gradient of Re <g5 xi_s | sgn(H) | xi_s>, the
 * eigenpairs' motion included (as tslov_sign_grad_batched_deflated computes it), and
 * the Ward residual of the deflated samples.  defl = NULL or l = 0 is
 * tslov_current_estimate.  Workspace: per source one link gradient and (for the Ward
 * check) three canonical spinors beyond tslov_sign_grad_batched_deflated's. */
tslov_status tslov_current_estimate_deflated(tslov_ctx* ctx, int nsrc, const void* xi, const int* k,
                                             const tslov_deflation* defl, double* j_out, double* div_out,
                                             double* tot_out, double* ward_out, tslov_info* infos);

/* Solve with the overlap operator (Sec. 1 eq. overlap, a = 1): x = D_ov^{-1} b
 * (adjoint = 0) or x = D_ov^{-dag} b (adjoint = 1), with D_ov = 1 + g5 sgn(H) and sgn(H)
 * the context's two-sided Lanczos approximation of size k (no deflation), and
 * D_ov^dag = g5 D_ov(-mu) g5 (sgn(H)^dag = sgn(H(-mu))).  Conjugate gradients on the
 * normal equations, each iteration two approximate applications, stopped at
 * |b - A x| <= tol |b|.  The approximation is linear in its source only as far as it
 * has converged (eps_A), so tol below eps_A is not reachable.  b, x: canonical
 * spinors (device, distinct).  iters_out, relres_out (host, nullable): iterations and
 * the final relative residual.  ERR_NOT_CONVERGED when maxit iterations do not reach
 * tol (x holds the last iterate). */
tslov_status tslov_overlap_solve(tslov_ctx* ctx, const void* b, void* x, int k, int adjoint, double tol, int maxit,
                                 int* iters_out, double* relres_out);

/* The physical U(1) vector current of Sec. 4.3 eq. lat_vec_cur,
 *   j(x, nu) = Tr(D_ov^{-1} dD_ov/dTheta_{x,nu}),   U_nu(x) -> e^{i Theta} U_nu(x),
 * by the Z2-noise estimator over the nsrc sources xi ([nsrc][V][4][3], device):
 *   j_N = (1/N) sum_s chi_s^dag dD_ov/dTheta xi_s,   chi_s = D_ov^{-dag} xi_s
 * (tslov_overlap_solve with tol, maxit per source; the derivative through the TSL
 * approximation of size k, as tslov_sign_grad).  j_out (device): 8V doubles, the real
 * parts [4][V] then the imaginary parts [4][V] (direction x, y, z, t, site);
 * div_out, tot_out (device, nullable): 2V doubles each (real [V], imaginary [V]),
 * the divergence and total current of eq. divergence_def at every site.
 * iters_out, relres_out (host, nullable, nsrc): the solves' iterations and residuals.
 * Meaningful where the TSL approximation has converged (eps_A well below tol). */
tslov_status tslov_physical_current(tslov_ctx* ctx, int nsrc, const void* xi, int k, double tol, int maxit,
                                    double* j_out, double* div_out, double* tot_out, int* iters_out,
                                    double* relres_out);

/* A-posteriori error estimate (Sec. 4.1, eq. error_est): with y = TSL(psi) and
 * z = TSL(y) (a fresh Krylov space with source y, same k and deflation),
 * eps_A = |z - psi| / (2 |psi|).  eps_out: host double. */
tslov_status tslov_error_estimate(tslov_ctx* ctx, const void* psi, int k, const tslov_deflation* defl,
                                  double* eps_out);

/* The projected matrix of the two-sided Lanczos process on its own (Sec. 2):
 * T_out (host, k x k complex128, row-major) receives T_k with diagonal alpha_j,
 * T_{j+1,j} = beta_{j+1} and T_{j,j+1} = gamma_{j+1} for j < k_used; rows and
 * columns past k_used are zero.  Its eigenvalues are the Ritz values whose signs
 * the approximation interpolates (diagnostics: min |Re theta|). */
tslov_status tslov_lanczos_matrix(tslov_ctx* ctx, const void* psi, int k, void* T_out, tslov_info* info);

/* The small dense step of the method on its own (Sec. 2, eq. spectral_form applied to
 * the projected matrix): c_out = sgn(T) e_1 for the k x k complex tridiagonal T with
 *   T_jj = diag[j] (k complex), T_{j+1,j} = sub[j] (k-1 real), T_{j,j+1} = sup[j] (k-1 complex),
 * host arrays of interleaved (re, im) doubles; c_out: device, k complex128.  Runs the
 * same scaled Newton iteration as tslov_sign.  ERR_SIGN_UNDEFINED when an eigenvalue
 * of T has |Re| <= 1e-12 times the infinity norm of T (info->min_abs_re_ritz). */
tslov_status tslov_tridiag_sign(tslov_ctx* ctx, int k, const double* diag, const double* sub, const double* sup,
                                void* c_out, tslov_info* info);

/* Eigenvalues of the k x k complex tridiagonal T (same host arrays as
 * tslov_tridiag_sign) into out (host, 2k doubles, re/im), by the Ehrlich-Aberth
 * iteration on the characteristic polynomial's three-term recurrence (host code
 * only: needs no device and no context).  *sweeps (nullable) receives the sweeps
 * used, or -1 when some eigenvalue did not settle to rounding level. */
tslov_status tslov_ritz_values(int k, const double* diag, const double* sub, const double* sup, double* out,
                               int* sweeps);

/* The paper's derivative method (Sec. 2, Theorem 1 and eq. func_derivative_1) for one
 * link parameter t, U_nu(site) -> exp(i t X) U_nu(site) (X: host 3 x 3 complex
 * matrix, 18 doubles row-major re/im; the derivative is linear in X, and a
 * Hermitian traceless X is an su(3) direction, X = 1 the U(1) phase): the
 * two-sided Lanczos process of size k on the block matrix
 *   B = [[H, dH], [0, H]],   dH = d H / dt,
 * from the source (x1, x2) (canonical spinors, device; x1 = NULL means zero), both
 * Krylov spaces of B started there, y = |x| V_B sgn(T_B) e_1 with the halves into
 * y1_out and y2_out.  With x1 = NULL, y1_out approximates d sgn(H) x2 / dt and y2_out
 * sgn(H) x2 (eq. func_derivative_1); this differs at finite k from the derivative of
 * the k-step approximation that tslov_sign_grad returns (it equals the derivative of
 * the Ritz interpolation polynomial with its coefficients held fixed).  Float64
 * whatever the context precision; the context's links and mu.  ERR_ARG for a link
 * out of range or a non-finite X; ERR_BREAKDOWN as tslov_sign. */
tslov_status tslov_block_sign(tslov_ctx* ctx, int nu, int site, const double* X, const void* x1, const void* x2,
                              int k, void* y1_out, void* y2_out, tslov_info* info);

/* The block-matrix process deflated by eigenpairs of H (App. E, eq. array_app_defl_1):
 * the eigenpairs (lambda_i, R_i, L_i) of defl (as for tslov_sign; L^H R = 1, distinct
 * eigenvalues, accurate for the links set) span with their derivatives the
 * 2l-dimensional invariant subspace of B with right basis (R_i, 0), (dR_i, R_i), which
 * is treated exactly:
 *   y = sum_i s_i [(R_i, 0) c1_i + (dR_i, R_i) c2_i] + TSL_k(B, Pbar x),
 *   c2_i = L_i^H x2,  c1_i = L_i^H x1 + <dL_i|x2>,  s_i = sgn Re lambda_i,
 *   Pbar x = (x1 - sum_i (c1_i R_i + c2_i dR_i), x2 - sum_i c2_i R_i),
 * every coefficient taken from the input.  The eigenvector derivatives (normalised
 * <L_i|dR_i> = <dL_i|R_i> = 0, eq. c1i_3 and eq. dRi) need the 2l singular
 * consistent systems (lambda_i - H) z = P dH R_i and (lambda_i - H) z = P x2
 * (P = 1 - sum_j R_j L_j^H), solved on the device by conjugate gradients on the
 * normal equations to relative residual 1e-13 (ERR_NOT_CONVERGED after 1e5
 * iterations; info->cg_iters = iterations used), their R_i components removed.
 * defl = NULL or l = 0 is tslov_block_sign.  Other arguments and errors as there. */
tslov_status tslov_block_sign_deflated(tslov_ctx* ctx, int nu, int site, const double* X, const void* x1,
                                       const void* x2, int k, const tslov_deflation* defl, void* y1_out,
                                       void* y2_out, tslov_info* info);

/* Its error estimate (Sec. 4.1 eq. bA_error_est): with (y1, y2) = TSL_k(B, (0, psi))
 * and (z1, z2) = TSL_k(B, (y1, y2)) (a fresh process from the first result),
 * eps_B = |(z1, z2 - psi)| / (2 |psi|).  eps_out: host double. */
tslov_status tslov_block_error_estimate(tslov_ctx* ctx, int nu, int site, const double* X, const void* psi, int k,
                                        double* eps_out);

/* eps_B with the deflated block process (tslov_block_sign_deflated) for both
 * applications, the second from the first result (App. E: the reason for deflating
 * general sources).  defl = NULL or l = 0 is tslov_block_error_estimate. */
tslov_status tslov_block_error_estimate_deflated(tslov_ctx* ctx, int nu, int site, const double* X, const void* psi,
                                                 int k, const tslov_deflation* defl, double* eps_out);

/* One link parameter of the block-matrix derivative: U_nu(site) -> exp(i t X) U_nu(site),
 * X a 3 x 3 complex matrix as 18 doubles, row-major (re, im). */
typedef struct {
    int nu;
    int site;
    double X[18];
} tslov_link_direction;

/* The tuning run that fixes the Krylov sizes before production runs (Sec. 4.1,
 * numerical setup and tuning).  The trial vector is phi = (1, ..., 1) (built here).
 * For every candidate i (outer size k_outer[i], nested inner size k_inner[i], 0 for
 * the plain step; k_inner may be NULL for all-plain candidates):
 *   eps_out[i] = eps_A of eq. error_est of the (deflated, if defl) sign of phi, or,
 *                with dir, eps_B of eq. bA_error_est for that link direction and the
 *                sparse source (0, phi), of the deflated block process if defl
 *                (tslov_block_error_estimate_deflated; k_inner must be 0 then);
 *   ms_out[i]  = wall time in ms of the first approximation (the sign of phi, or the
 *                first block process), taken on its second run so that allocation and
 *                first touch of a larger workspace do not count.
 * A candidate whose process breaks down seriously or whose projected matrix has a
 * Ritz value on the imaginary axis gets eps = +inf and ms = NaN.  *chosen receives the
 * fastest candidate with eps <= trial_target (the first of equal times), -1 if none;
 * the paper's rule of thumb is trial_target = 0.1 eps_0 for a wanted precision eps_0.
 * With nrand > 0 and a choice, cross_out[r] receives the same error estimate for the
 * caller's vector r of rand ([nrand][V][4][3] complex128, device) at the chosen
 * parameters (the paper's cross-check, 20-30 random vectors, compared with eps_0 by
 * the caller).  The context's nested setting is unchanged on return.  Times depend on
 * the machine, so *chosen may differ between runs where candidates take similar time.
 * ERR_ARG for sizes out of range, a bad direction, or nested block mode. */
tslov_status tslov_tune_k(tslov_ctx* ctx, int ncand, const int* k_outer, const int* k_inner, double trial_target,
                          const tslov_deflation* defl, const tslov_link_direction* dir, int nrand, const void* rand,
                          double* eps_out, double* ms_out, int* chosen, double* cross_out);

/* Nested projected-matrix step (one level of nesting, the paper's production
 * setting, Sec. 4.1; the nested method itself is cited there, not described).
 * With k_inner = m > 0, tslov_sign, tslov_overlap and tslov_error_estimate replace
 * the dense sgn(T_k) e_1 of the outer process (k = k_used > m) by
 *   T_k W^{1/2} e_1 ~ T_k V' (T')^{1/2} e_1,   W = (T_k^2)^{-1},
 * an inner two-sided Lanczos process of size m on W with both spaces started from
 * e_1 (its basis V', its projected matrix T', the principal square root).  The
 * identity z (z^2)^{-1/2} = sgn(Re z) makes it exact for m = k; the inner space
 * resolves the eigenvalues of T_k nearest zero first, so m well below k suffices
 * (m = 100 is the paper's inner size).  The dense work then is O(k^2 m) for W and
 * the inner products plus O(m^3) for the square root, in place of O(k^3) Newton
 * steps.  k_inner = 0 (the default) or k_inner >= k_used: the plain dense step.
 * The derivative calls always use the plain step (their Frechet derivative is that
 * of sgn(T_k)).  ERR_ARG for k_inner outside [0, 1024]; ERR_BREAKDOWN for a serious
 * breakdown of the inner process. */
tslov_status tslov_set_nested(tslov_ctx* ctx, int k_inner);

/* Optional per-call diagnostics of the context: TSLOV_DIAG_EPS_A makes tslov_sign,
 * tslov_overlap and tslov_sign_grad compute info->eps_A (Sec. 4.1 eq. error_est: one
 * more two-sided Lanczos process of size k on the output; only when info is given).
 * flags = 0 turns them off (the default).  ERR_ARG for unknown bits. */
#define TSLOV_DIAG_EPS_A 1
tslov_status tslov_set_diagnostics(tslov_ctx* ctx, int flags);

/* Projected-matrix step on its own (for tests): S = sgn(T) for a dense complex128
 * k x k row-major device matrix T by the scaled Newton iteration, and, if E is
 * not NULL, L = L_sgn(T, E), the upper-right block of sgn([[T, E], [0, T]])
 * (Theorem 1).  S_out, L_out: device k x k; iters (host, nullable). */
tslov_status tslov_dense_sign(tslov_ctx* ctx, const void* T, int k, const void* E,
                              void* S_out, void* L_out, int* iters);

/* Kernel timing for roofline measurement.  With every = N >= 1 the library records
 * a HIP event pair around every N-th launch of each kernel class on its stream
 * (every = 0 turns timing off; each pair adds a few microseconds of dispatch
 * latency to the stream, so a sparse sample perturbs the timed work least).
 *   which = 0: forward Lanczos stencil pair (the dominant kernel)
 *   which = 1: backward stencil pair
 *   which = 2: plain operator application (tslov_apply_dw / tslov_apply_h)
 * tslov_timing_read synchronises the stream and returns the number of timed
 * launches and their summed duration, then clears the record. */
tslov_status tslov_timing_enable(tslov_ctx* ctx, int every);
tslov_status tslov_timing_read(tslov_ctx* ctx, int which, int* count, double* total_ms);

/* Captured iteration loops.  With on = 1 the forward and reverse Lanczos loops of
 * the derivative and sign calls (two launches per step each) are captured as HIP
 * graphs on first use and replayed by later calls with the same source sizes,
 * workspace and launch shapes; anything else recaptures.  Results are identical
 * to the launched loops.  Capture is skipped while kernel timing is on, while
 * the batched pair-kernel shape is still being timed and in recompute mode.
 * Needs a context created on a non-null stream (ERR_ARG otherwise); the stream
 * must not be captured by the caller.  on = 0 (the default) frees the graphs. */
tslov_status tslov_set_graphs(tslov_ctx* ctx, int on);

/* Launch shape of the operator (tslov_apply_dw / tslov_apply_h) on lattices whose
 * t-slices split into whole tiles of 128 sites over the 8 XCDs (e.g. 32^4): each
 * thread marches through T consecutive t-slices.  T = 0 (the default) lets the
 * first call time the candidates (divisors of N_t giving 128 to 4096 workgroups,
 * best of three launches each) and keep the fastest for the context; T > 0
 * forces that chunk length.  Results do not depend on T.  ERR_ARG unless T = 0
 * or T divides N_t (the value is ignored where the operator does not march).
 * tslov_get_apply_chunk returns the timed pick (0 while none is made or where
 * the operator does not march). */
tslov_status tslov_set_apply_chunk(tslov_ctx* ctx, int T);
tslov_status tslov_get_apply_chunk(const tslov_ctx* ctx, int* T);

/* Launch shape of the batched stencil pair kernels on lattices of more than 128
 * blocks of 64 sites (the colour-split layout): ns entries of a batch per
 * workgroup, which share every link load.  ns = 0 (the default) lets the library
 * time 1, 2 and 4 on the first steps of a batched call and keep the fastest for
 * the context's later calls; ns = 1, 2 or 4 forces that value (fewer when a
 * launch has fewer entries).  Results do not depend on it: each entry's
 * arithmetic is the same for every ns.  ERR_ARG for any other ns.
 * tslov_get_pair_ns returns the timed picks (0 while none is made) of the
 * forward (fwd_ns) and reverse (bwd_ns) kernels; either pointer may be NULL. */
tslov_status tslov_set_pair_ns(tslov_ctx* ctx, int ns);
tslov_status tslov_get_pair_ns(const tslov_ctx* ctx, int* fwd_ns, int* bwd_ns);

/* Operator form of the shifted solves in the deflated derivative (the conjugate
 * gradients on the normal equations of the 2l systems (lambda_i - H) z = ...,
 * Sec. 3 with App. B), each application covering all unconverged systems:
 *   form = 0: multi-right-hand-side, eight systems per wavefront at eight sites,
 *            reading each link element in one load;
 *   form = 1: colour split, two systems per workgroup;
 *   form = 2: the multi-right-hand-side layout with the link times half-spinor
 *            products on the float64 matrix cores (v_mfma_f64_16x16x4f64);
 *   form = 3 (the default): each thread marches one (x, y, z) site of one system
 *            along t, the systems of a tile running back to back on one XCD.
 * The results agree to rounding (the forms differ in the summation order of the
 * residual norms and, on the matrix cores, of the link products).  Form 3 needs an
 * (x, y, z) volume in multiples of 1024 sites and runs form 0 otherwise; forms 0
 * and 2 need 7 * 5 * 12 * ldv + ldv complex doubles to stay below 4 GiB (lattices
 * up to about 639,000 sites) and run form 1 above that.  ERR_ARG for any other
 * form. */
tslov_status tslov_set_cg_operator(tslov_ctx* ctx, int form);

/* Algorithmic bytes moved by one launch of kernel class `which` (see above) for
 * this context's lattice and precision (minimal traffic, each field once). */
double tslov_kernel_bytes(const tslov_ctx* ctx, int which);

#ifdef __cplusplus
}
#endif
#endif /* TSLOV_H */
