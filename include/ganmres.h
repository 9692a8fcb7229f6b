/*
 * ganmres.h - C ABI of the MI355X (gfx950) GA-NGMRES transport-registration
 * library (libganmres.so).
 *
 * The library evaluates, on one GPU, the reduced objective and gradient of
 * the transport-constrained optimal control problem of He & Mang, "A
 * generalized alternating NGMRES method for PDE-constrained optimization
 * problems governed by transport equations" (eq. e:varopt and, for
 * mass-preserving transport, eq. e:varopt-optimal-transport), the spectral
 * preconditioner of the fixed-point map (eq. e:rpgd), and one iteration of
 * GA-NGMRES (Alg. 3) around that map.
 *
 * Conventions shared by every call:
 *   - Return value: GANMRES_OK (0) or a negative GANMRES_E* code.  Nothing is
 *     thrown across the ABI; ganmres_last_error() describes the last failure
 *     of a handle (static lifetime until the next call on that handle).
 *   - Arrays are DEVICE pointers owned by the caller, contiguous C order.
 *     A scalar field ("image") has shape (n[0], .., n[dim-1]) - the last axis
 *     contiguous; a vector field ("velocity") has shape (dim, n[0], ..,
 *     n[dim-1]), component c acting along axis c.  The element type is float
 *     (GANMRES_F32) or double (GANMRES_F64) as chosen in the config.
 *   - Scalars returned to the host are written through HOST pointers; calls
 *     that return host scalars synchronise the handle's stream.
 *   - All device work is enqueued on the stream given to ganmres_create (a
 *     hipStream_t; NULL means the default stream).  One handle per stream;
 *     a handle is not thread-safe.
 *   - The library owns only its workspace, allocated in ganmres_create (and,
 *     for the solver history and the next direction's spectrum, during the
 *     first ganmres_step) and released by ganmres_destroy.
 *
 * Discretisation (Sec. 2.2): periodic box [0,2pi)^dim, n_i cells of size
 * h_i = 2 pi / n_i, Fourier pseudo-spectral derivatives, semi-Lagrangian time
 * stepping with n_t steps of h_t = 1/n_t and an explicit RK2 backtrace, cubic
 * Lagrange (tricubic / bicubic) interpolation at departure points, trapezoidal
 * rule in time.  Grid sizes must be of the form 2^a 3^b with 4 <= n_i <= 1024.
 */
#ifndef GANMRES_H
#define GANMRES_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GANMRES_OK = 0,
    GANMRES_EINVAL = -1,       /* invalid argument or configuration          */
    GANMRES_ENOMEM = -2,       /* device allocation failed                   */
    GANMRES_EDEVICE = -3,      /* a HIP call failed                          */
    GANMRES_ENONFINITE = -4,   /* NaN/Inf in an objective, gradient or norm  */
    GANMRES_ELINESEARCH = -5,  /* Armijo condition not met in max_backtracks */
    GANMRES_ELSQ = -6,         /* least-squares coefficients not finite      */
    GANMRES_ESTATE = -7        /* call out of order (e.g. nothing to reuse)  */
};

enum { GANMRES_ADVECTION = 0, GANMRES_CONTINUITY = 1 };
enum { GANMRES_F32 = 0, GANMRES_F64 = 1 };
enum { GANMRES_VARIANT_GA = 0, GANMRES_VARIANT_ALT = 1 };
enum { GANMRES_STEP_NGMRES = 0, GANMRES_STEP_FP = 1, GANMRES_STEP_AA = 2, GANMRES_STEP_NEWTON = 3 };
enum { GANMRES_ACCEL_NGMRES = 0, GANMRES_ACCEL_AA = 1, GANMRES_ACCEL_NK = 2 };
enum { GANMRES_PC_IREG = 0, GANMRES_PC_H0RPC = 1, GANMRES_PC_2LRPCSYM = 2 };

typedef struct ganmres_handle ganmres_handle;

typedef struct {
    int dim;               /* 2 or 3                                            */
    int n[3];              /* grid cells per axis (first dim entries used)      */
    int nt;                /* time steps, >= 1                                  */
    int model;             /* GANMRES_ADVECTION (eq. e:varopt) or
                              GANMRES_CONTINUITY (eq. e:varopt-optimal-transport) */
    int incompressible;    /* 1: Leray-projected gradient (Sec. 3.5)            */
    int reg_order;         /* p in 1..3: l_p(k) = |k|^(2p) (H1, H2, H3 models)  */
    double alpha;          /* regularisation weight, > 0                        */
    int dtype;             /* GANMRES_F32 or GANMRES_F64                        */
    int checkpoint_every;  /* keep every c-th state of the forward history (>=1) */
} ganmres_config;

typedef struct {
    int w;                 /* window depth, >= 0 (w_k = min(k, w))              */
    int sigma;             /* NGMRES steps per cycle, >= 0 (0: plain FP / RPGD) */
    int tau;               /* fixed-point steps per cycle, >= 0                 */
    double eps_rel;        /* stop when ||g||_inf <= eps_rel ||g(v^0)||_inf     */
    int n_iter;            /* stop after n_iter updates                         */
    double c_armijo;       /* Armijo constant (paper: 1e-4)                     */
    int max_backtracks;    /* halvings before GANMRES_ELINESEARCH (e.g. 30)     */
    double rho_cap;        /* cap on the stored step, <= 0 means none           */
    int variant;           /* GANMRES_VARIANT_GA: FP when mod(k,s+t) >= sigma;
                              GANMRES_VARIANT_ALT: FP when mod(k,s+t) < tau     */
    int accel;             /* GANMRES_ACCEL_NGMRES (Alg. 1/3), GANMRES_ACCEL_AA
                              (Anderson acceleration, Alg. 2, with the same
                              alternation: GA-AA) or GANMRES_ACCEL_NK (the
                              Gauss-Newton-Krylov baseline, Appendix A; w,
                              sigma, tau, variant and rho_cap unused)           */
    int nk_precond;        /* GANMRES_ACCEL_NK: preconditioner of the Newton
                              step, GANMRES_PC_IREG ((alpha L)^-1),
                              GANMRES_PC_H0RPC or GANMRES_PC_2LRPCSYM (see
                              ganmres_newton_precond)                           */
} ganmres_solver_params;

#define GANMRES_MAX_WINDOW 64

typedef struct {
    int k;                 /* iterations completed after this call              */
    int step_kind;         /* GANMRES_STEP_NGMRES, _AA, _FP or _NEWTON          */
    int stop;              /* 1 when the stopping rule of Alg. 3 holds          */
    int n_trials;          /* objective evaluations in this line search         */
    int n_grad;            /* gradient evaluations in this call                 */
    int n_beta;            /* number of valid entries in beta (Newton steps:
                              the CG iterations taken)                          */
    int lsq_fallback;      /* 1 when this step's least-squares solve fell back
                              from Cholesky to the pseudo-inverse (rank-deficient
                              or ill-conditioned window, see ganmres_lsq)       */
    double J;              /* J(v^{k+1})                                        */
    double J_q;            /* J(q(v^k))                                         */
    double ginf;           /* ||g(v^{k+1})||_inf                                */
    double g0inf;          /* ||g(v^0)||_inf                                    */
    double rho;            /* accepted step                                     */
    double beta[GANMRES_MAX_WINDOW + 1];
} ganmres_step_info;

/* Create a problem for template m0 and reference m1 (device images of cfg's
 * shape and dtype; both are copied).  stream: hipStream_t or NULL.
 * Errors: GANMRES_EINVAL (dim not 2/3, n_i not 2^a 3^b in [4,1024], nt < 1,
 * alpha <= 0, reg_order not 1..3, model/dtype unknown, incompressible with the
 * continuity model, checkpoint_every < 1), GANMRES_ENOMEM, GANMRES_EDEVICE. */
int ganmres_create(const ganmres_config* cfg, const void* m0, const void* m1,
                   void* stream, ganmres_handle** out);

/* A batch: count (1..64) independent 2-D problems of the same shape and
 * model in one handle, stacked along a leading axis, so that every kernel
 * launch serves all of them (the small-image regime, where one problem cannot
 * fill the GPU).  cfg describes one problem (dim must be 2 when count > 1);
 * alpha: host array of count regularisation weights (NULL: cfg->alpha for
 * all).  m0, m1: device images of shape (count, n[0], n[1]).  On a batch
 * handle a velocity has shape (2, count, n[0], n[1]) (component-major: all
 * problems' first components, then all second components); the evaluation
 * calls return sums over the problems (ganmres_batch_values gives them one
 * by one), and ganmres_step advances every problem by one iteration, each with
 * its own line search, window and mixing coefficients.  The problems share the
 * iteration counter k, so the GA switch of Alg. 3 is common; a problem whose
 * stopping rule holds keeps iterating until the caller stops.  A single
 * handle is the batch of one.  Errors: as ganmres_create, and GANMRES_EINVAL
 * for count outside [1, 64], count > 1 with dim 3, or alpha[i] <= 0. */
int ganmres_create_batch(const ganmres_config* cfg, int count, const double* alpha,
                         const void* m0, const void* m1, void* stream, ganmres_handle** out);

/* A group: batches of 2-D problems of DIFFERENT grid sizes in one handle
 * (uneven-size registrations, e.g. 16 problems each at 96^2, 192^2 and
 * 384^2), run so that every phase of an evaluation or iteration is one
 * kernel launch for all of them.  Class c (0 <= c < nclass <= 16) holds
 * counts[c] (1..64) problems of shape (shapes[2c], shapes[2c+1]); cfg gives
 * everything else (dim must be 2; cfg->n is ignored).  alpha: host array of
 * one weight per problem, classes in order (NULL: cfg->alpha for all).
 * m0[c], m1[c]: device images of shape (counts[c], shapes[2c], shapes[2c+1]).
 * On a group handle a velocity is the classes' batch velocities back to back,
 * class c's of shape (2, counts[c], shapes[2c], shapes[2c+1]) (see
 * ganmres_create_batch), and an image the classes' stacked images back to
 * back; per-problem results (ganmres_step's info, ganmres_batch_values,
 * ganmres_deformation's stats) list the problems class by class.  Each
 * problem has its own line search, window and mixing coefficients, as in a
 * batch; the classes backtrack together (a class whose problems have all
 * accepted waits) and take the same gather variant (the largest bound).  The
 * Newton-Krylov baseline (accel = GANMRES_ACCEL_NK), ganmres_hessian_matvec
 * and ganmres_newton_precond are not available on a group (GANMRES_EINVAL);
 * kernel timing has no effect.  Errors: as ganmres_create_batch, and
 * GANMRES_EINVAL for nclass outside [1, 16] or dim != 2. */
int ganmres_create_group(const ganmres_config* cfg, int nclass, const int* shapes,
                         const int* counts, const double* alpha, const void* const* m0,
                         const void* const* m1, void* stream, ganmres_handle** out);

/* Kernel launches of a group handle since its creation: *submitted counts the
 * launches its classes made, *issued the merged launches that ran them.
 * Errors: GANMRES_EINVAL (not a group handle). */
int ganmres_group_launches(const ganmres_handle* h, long long* submitted, long long* issued);

/* The 2-D tile autotuner: the semi-Lagrangian kernels of a 2-D handle run on
 * tiles of 64 x 4P points with P = 8, 4 or 2 points per thread, chosen when
 * the handle (or each class of a group) is created by timing the gather step
 * of every variant on its grid, once per grid size and element type in the
 * process.  Reports class cls's choice (cls = 0 for a handle that is not a
 * group): *points_per_thread = P (0 for a 3-D handle, which has no variants)
 * and, in us (host, nullable, 3 entries), the measured microseconds per
 * gather launch of P = 8, 4, 2.  Errors: GANMRES_EINVAL. */
int ganmres_tile_autotune(const ganmres_handle* h, int cls, int* points_per_thread, double* us);

/* Number of problems in the handle (1 for ganmres_create; 0 for NULL). */
int ganmres_batch_count(const ganmres_handle* h);

/* Per-problem J and 1/2 ||m(1) - m1||_h^2 of the last objective or gradient
 * evaluation (host arrays of ganmres_batch_count entries, either nullable). */
int ganmres_batch_values(ganmres_handle* h, double* J, double* mismatch);

/* Release the handle and its workspace (NULL is accepted). */
int ganmres_destroy(ganmres_handle* h);

/* Message for the last failure on h (or, if h is NULL, of the last failed
 * call without a handle on this thread: ganmres_create,
 * ganmres_create_batch, ganmres_eval_objective_noalloc). */
const char* ganmres_last_error(const ganmres_handle* h);

/* Objective J(v) = 1/2 ||m(1) - m1||_h^2 + alpha/2 <v, L_p v>_h (eq. e:varopt;
 * <a,b>_h = prod(h_i) sum a b).  v: device velocity.  J: host, required.
 * mismatch: host, nullable: 1/2 ||m(1) - m1||_h^2.
 * keep_history = 1 keeps the state history, departure points and spectra
 * of v for a following ganmres_eval_gradient(..., reuse_forward = 1).
 * Errors: GANMRES_ENONFINITE. */
int ganmres_eval_objective(ganmres_handle* h, const void* v, int keep_history,
                           double* J, double* mismatch);

/* The objective of ganmres_eval_objective without a handle and without any
 * device allocation, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  cfg, m0,
 * m1 describe the problem as for ganmres_create (checkpoint_every must be 1);
 * v is the velocity.  m0, m1, v: device arrays owned by the caller; J: host,
 * required; mismatch: host, nullable; stream: hipStream_t or NULL.
 * Every intermediate field (the FP64 spectrum of v, the departure points, two
 * state fields, the window table, the divergence and source factor of the
 * continuity model, the FFT twiddles, the reduction partials) lives in one
 * static device array of 32 MiB per GPU, held until the process ends: about
 * (d + 2) N s + 16 d N_h + 0.5 MiB bytes (N points, N_h half-spectrum
 * points, s = 4 or 8; two more N s for the continuity model), e.g. 2-D grids
 * up to 512^2 and 3-D grids up to 64^3 in either precision.  A larger problem
 * is rejected with GANMRES_EINVAL (ganmres_last_error(NULL) gives the bytes
 * it needs) before any device work.  The call enqueues on the stream,
 * synchronises it twice (the window bound, the result) and calls no
 * allocating routine.  All calls on one GPU share the array: calls that
 * overlap in time on one GPU (other threads, other streams) race and must be
 * serialised by the caller.  Nothing in the array needs to start at zero
 * (each call writes every value it reads).
 * Errors: GANMRES_EINVAL, GANMRES_ENONFINITE, GANMRES_EDEVICE. */
int ganmres_eval_objective_noalloc(const ganmres_config* cfg, const void* m0, const void* m1,
                                   const void* v, void* stream, double* J, double* mismatch);

/* Reduced gradient g(v) = alpha L_p v + b (eq. e:reduced-gradient) with
 * b = int lam grad m dt (advection, adjoint eq. e:adjoint with final value
 * lam(1) = m1 - m(1)), b = -int pi grad lam dt (continuity), and b replaced
 * by its Leray projection when incompressible.  g is the L2 representer: a
 * grid function with dJ(v)[d] ~ <g, d>_h.  v, g: device velocities (may not
 * alias).  reuse_forward = 1: the caller asserts that the last evaluation on
 * the handle (ganmres_eval_objective(keep_history = 1) or
 * ganmres_eval_gradient) was for this same v, unchanged since, and its forward
 * solve is reused.  J: host, nullable.
 * Errors: GANMRES_ESTATE (reuse without a kept history), GANMRES_ENONFINITE. */
int ganmres_eval_gradient(ganmres_handle* h, const void* v, void* g,
                          int reuse_forward, double* J);

/* Search direction of the preconditioned fixed-point map (eqs. e:rpgd,
 * e:fixedpoint): s = -(alpha L_p)^-1 g, the zero symbol entry replaced by
 * one (Sec. 2.2), Leray-projected when incompressible.  g, s: device
 * velocities (may alias).  gs: host, nullable: <g, s>_h. */
int ganmres_apply_precond(ganmres_handle* h, const void* g, void* s, double* gs);

/* One iteration k of GA-NGMRES(w; sigma, tau) (Alg. 3), or of GA-AA with
 * accel = GANMRES_ACCEL_AA (Alg. 2 with the alternation of Alg. 3), around the
 * line-searched map q(v) = v + rho s (eqs. e:linesearch, e:armijo).  v: device
 * velocity, in: v^k, out: v^{k+1}.  On the first call after create or reset, v
 * is v^0 and g(v^0) is evaluated first.  The handle keeps k, the stored step
 * rho, the window (the last w+1 pairs (v, g), or the last w pairs
 * (v - q(v), q(v)) for AA) and ||g(v^0)||_inf.  info: host array of
 * ganmres_batch_count(h) entries (one per problem), nullable.
 * With accel = GANMRES_ACCEL_NK the call is one inexact Gauss-Newton-Krylov
 * iteration instead (Appendix A): preconditioned CG on H_gn s = -g (see
 * ganmres_hessian_matvec) with the preconditioner (alpha L_p)^-1, stopped when
 * ||r||_h <= min(1/2, sqrt(||g||_h / ||g(v^0)||_h)) ||g||_h or after 50
 * iterations, then Armijo backtracking from rho = 1 (advection model, full
 * history, single problem); p->nk_precond selects the preconditioner.
 * Errors: GANMRES_EINVAL (w < 0 or > GANMRES_MAX_WINDOW, sigma = tau = 0,
 * negative counts, unknown accel, accel or w changed without a reset,
 * GANMRES_ACCEL_NK outside its setting), GANMRES_ELINESEARCH, GANMRES_ELSQ,
 * GANMRES_ENONFINITE. */
int ganmres_step(ganmres_handle* h, const ganmres_solver_params* p, void* v,
                 ganmres_step_info* info);

/* Transport map and its Jacobian determinant, the diffeomorphism check shown
 * with the paper's results (Sec. 3; Sec. 3.5 reports det grad y = 1 for
 * incompressible flows as min, mean, max and standard deviation).  y is the
 * foot at t = 0 of the characteristic through x at t = 1, m(1) = m0 o y,
 * built with the state's semi-Lagrangian steps: y = x + h D,
 *   D^0 = 0,  D^{j+1}(i) = (X_i - i) + I[D^j](X_i)   (cells, X the RK2
 * departure points of v), and grad y = Id + (h_a dD_a/dx_b) with spectral
 * derivatives.  v: device velocity.  det: device image (nullable) receiving
 * det grad y.  stats: host array of 4 doubles per problem (see
 * ganmres_batch_count): min, mean, max, standard deviation of det grad y.
 * The call replaces the handle's departure points, so a following
 * ganmres_eval_gradient(reuse_forward = 1) needs a new objective evaluation.
 * Errors: GANMRES_ENONFINITE. */
int ganmres_deformation(ganmres_handle* h, const void* v, void* det, double* stats);

/* Gauss-Newton Hessian matvec of the Newton-Krylov baseline (Appendix A,
 * eqs. e:hessian-matvec, e:incremental-state, e:incremental-adjoint with the
 * terms carrying lam dropped):
 *   out = H_gn[v] vt = alpha L_p vt + [P] int lt grad m dt,
 * with the incremental state mt (mt(0) = 0, source -vt . grad m) integrated
 * along the state's characteristics by the trapezoidal rule, and lt solving
 * the adjoint equation with final value -mt(1).  v, vt, out: device
 * velocities; out may alias neither.  The state of v is solved again on every
 * call.  The advection model with the full state history on a single
 * problem only.  The call replaces the handle's adjoint fields.
 * Errors: GANMRES_EINVAL (continuity model, checkpoint_every > 1, a batch). */
int ganmres_hessian_matvec(ganmres_handle* h, const void* v, const void* vt, void* out);

/* Apply a preconditioner of the Newton step at velocity v (Appendix A,
 * "Preconditioning"): z = M^-1 r.  which:
 *   GANMRES_PC_IREG      M = alpha L_p ([P] when incompressible);
 *   GANMRES_PC_H0RPC     M = H0, the Gauss-Newton Hessian at v = 0,
 *                        H0 z = alpha L z + [P] grad m0 (grad m0 . z), inverted
 *                        by GMRES on (alpha L)^-1 H0 z = (alpha L)^-1 r;
 *   GANMRES_PC_2LRPCSYM  two-level: the low band of the symmetric
 *                        regularisation-preconditioned Hessian
 *                        I + Hreg^-1/2 H_data Hreg^-1/2 (Hreg = alpha L),
 *                        discretised on the grid with half the cells per axis
 *                        (images and v restricted spectrally, the coarse
 *                        Nyquist modes dropped) and inverted by CG there; the
 *                        high band takes Hreg^-1:
 *                        z = prolong(Hreg^-1/2 y) + P_hf Hreg^-1 r.
 * The inner solves stop at a relative residual of 1e-1 or after 10
 * iterations (the Newton-Krylov iteration of ganmres_step uses the flexible
 * CG update with the last two).  v, r, z: device velocities, z aliasing
 * neither.  The advection model with the full state history on a single
 * problem; 2LRPCSYM needs even sizes of at least 8.  The call replaces the
 * handle's adjoint fields.
 * Errors: GANMRES_EINVAL. */
int ganmres_newton_precond(ganmres_handle* h, int which, const void* v, const void* r, void* z);

/* The least-squares problem of the NGMRES mixing step (Alg. 1, and Alg. 3's
 * NGMRES iterations): beta = argmin || r + sum_i beta_i (r - g_i) ||_2 over
 * the columns of the window, from the Gram matrix of u = [r, g_0, ..,
 * g_{K-2}] (G: host, K x K row major, symmetric, finite; 2 <= K <= 66).
 * With M_ij = (r - g_i).(r - g_j) the normal equations M beta = -(|r|^2 -
 * r.g_i) are solved by Cholesky; when it breaks down or the squared pivot
 * ratio is below 1e-12 (the window is rank-deficient or nearly so; Sec. 2.3
 * leaves the treatment of rank deficiency open), by the eigen pseudo-inverse
 * with cutoff 1e-12 lambda_max.  This is the host solve ganmres_step uses.
 * beta: host, K - 1 entries.  fallback: host, nullable, set to 1 when the
 * pseudo-inverse was used.  Errors: GANMRES_EINVAL, GANMRES_ELSQ. */
int ganmres_lsq(int K, const double* G, double* beta, int* fallback);

/* Forget the solver state (k, rho, history); the next ganmres_step starts a
 * new solve from the v it is given. */
int ganmres_solver_reset(ganmres_handle* h);

/* Copy a field of the last forward/adjoint solve into out (device image):
 * which = 0: state m^j, which = 1: adjoint lam^j (j in 0..nt).  The state is
 * available after any objective or gradient evaluation, the adjoint after a
 * gradient evaluation.  Errors: GANMRES_EINVAL, GANMRES_ESTATE. */
int ganmres_get_field(ganmres_handle* h, int which, int j, void* out);

/* Kernel timing.  With on = 1 the library brackets every launch of the
 * selected kernel classes (all by default) with HIP events on its stream and
 * accumulates per-class device time.  ganmres_timing_select sets the classes
 * (bit k of mask: class k); an event pair costs the stream a few microseconds,
 * so a measurement that times one class should select only that one.  The
 * gathers of one forward or adjoint sweep run back to back and share one
 * event pair: they add their number of launches and the time of the sweep.
 * ganmres_timing_get returns the accumulated milliseconds and launch count of
 * class `kernel` (see ganmres_kernel_name) and the number of classes;
 * ganmres_timing_reset clears the accumulators. */
int ganmres_timing_enable(ganmres_handle* h, int on);
int ganmres_timing_select(ganmres_handle* h, unsigned mask);
int ganmres_timing_reset(ganmres_handle* h);
int ganmres_timing_get(ganmres_handle* h, int kernel, double* ms, long long* launches);
int ganmres_kernel_count(void);
const char* ganmres_kernel_name(int kernel);

/* Device bytes held by the handle's workspace. */
long long ganmres_workspace_bytes(const ganmres_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* GANMRES_H */
