// Runtime of the GA-NGMRES transport library: workspace, the reduced
// objective / gradient pipeline, the preconditioned fixed-point map with
// Armijo backtracking, and one GA-NGMRES iteration (the C ABI of ganmres.h).
#include <hip/hip_runtime.h>
#include <ucontext.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ganmres.h"
#include "config.hpp"
#include "fft_core.hpp"
#include "group.hpp"
#include "launch.hpp"

namespace gan {

// Kernel classes for the optional event timing.
enum KernelClass {
    KC_CHAR = 0,   // RK2 characteristics
    KC_SL,         // semi-Lagrangian gather step (state and adjoint)
    KC_FACTOR,     // source factors
    KC_DERIV,      // per-axis spectral derivative (body force, divergence)
    KC_RFFT,       // full forward transform
    KC_IRFFT,      // full inverse transform
    KC_SPEC,       // pointwise spectral operators
    KC_REDUCE,     // FP64 reductions (mismatch, dots, Gram, norms)
    KC_VEC,        // axpy / NGMRES update
    KC_COUNT
};
static const char* kKernelNames[KC_COUNT] = {"characteristics", "sl_step",    "source_factor",
                                             "deriv_axis",      "rfft",       "irfft",
                                             "spectral_op",     "reduction",  "vector_update"};

struct Status {
    int code = GANMRES_OK;
    std::string msg;
};

class Error {
   public:
    Error(int c, std::string m) : code(c), msg(std::move(m)) {}
    int code;
    std::string msg;
};

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::gan::Error(e_ == hipErrorOutOfMemory ? GANMRES_ENOMEM : GANMRES_EDEVICE, \
                               std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    void alloc(size_t b) {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (b == 0) return;
        HIPCHK(hipMalloc(&p, b));
        bytes = b;
    }
};

// ---- cooperative scheduler of group handles ----------------------------------
// The classes of a group handle (batches of different grid sizes) run their
// ordinary Problem code as cooperative tasks, each on its own stack
// (ucontext), all on the calling thread.  A task runs until it reaches a
// kernel launch (submit in group.hpp), a stream synchronisation or a group
// reduction, and hands that to the scheduler.  When every task waits, the
// scheduler issues all waiting launches, merging those of one family into
// one launch; synchronises the stream once when tasks wait for results and
// no launch is pending; and completes a reduction when every task has
// reached it.  A task's own operations stay in its program order, and the
// classes share no data, so the results are those of running the classes
// one after another.
struct CoopTask {
    enum State { RUN, LAUNCH, SYNC, BARRIER, DONE };
    ucontext_t ctx;
    ucontext_t* home = nullptr;
    std::unique_ptr<char[]> stack;
    State state = RUN;
    LaunchDesc desc;
    long long bval = 0;  // reduction: contribution in, result out
    int bop = 0;         // reduction operator: 0 max, 1 logical or
    int fail = 0;        // the awaited operation failed (fail_msg)
    std::string fail_msg;
    std::function<void()> fn;
    int err = GANMRES_OK;  // how the task's work ended
    std::string err_msg;
};

constexpr int kMaxClasses = 16;  // size classes of a group handle

struct CoopStats {
    long long submitted = 0;  // launches handed over by the tasks
    long long issued = 0;     // launches the scheduler made of them
};

static thread_local CoopTask* g_coop = nullptr;
CoopTask* coop_current() { return g_coop; }

static void coop_wait(CoopTask* t, CoopTask::State s) {
    t->state = s;
    g_coop = nullptr;
    swapcontext(&t->ctx, t->home);
    g_coop = t;
    if (t->fail) {
        t->fail = 0;
        throw Error(GANMRES_EDEVICE, t->fail_msg);
    }
}
void coop_launch(CoopTask* t, const LaunchDesc& d) {
    t->desc = d;
    coop_wait(t, CoopTask::LAUNCH);
}
static void coop_sync(CoopTask* t) { coop_wait(t, CoopTask::SYNC); }
static long long coop_reduce(CoopTask* t, long long v, int op) {
    t->bval = v;
    t->bop = op;
    coop_wait(t, CoopTask::BARRIER);
    return t->bval;
}

static void coop_entry(unsigned lo, unsigned hi) {
    CoopTask* t = reinterpret_cast<CoopTask*>((static_cast<uintptr_t>(hi) << 32) | lo);
    try {
        t->fn();
    } catch (const Error& e) {
        t->err = e.code;
        t->err_msg = e.msg;
    } catch (const std::bad_alloc&) {
        t->err = GANMRES_ENOMEM;
        t->err_msg = "host allocation failed";
    } catch (...) {
        t->err = GANMRES_EDEVICE;
        t->err_msg = "unexpected error";
    }
    t->state = CoopTask::DONE;
    g_coop = nullptr;  // uc_link resumes the scheduler
}

// Run fns[i] as cooperating tasks on stream st; rethrows the first task error.
static void coop_run(const std::vector<std::function<void()>>& fns, hipStream_t st, CoopStats* stats) {
    constexpr size_t kStack = size_t(1) << 20;
    const int n = static_cast<int>(fns.size());
    std::vector<std::unique_ptr<CoopTask>> tasks;
    ucontext_t home;
    for (int i = 0; i < n; ++i) {
        tasks.emplace_back(new CoopTask);
        CoopTask& t = *tasks.back();
        t.fn = fns[i];
        t.home = &home;
        t.stack.reset(new char[kStack]);
        if (getcontext(&t.ctx) != 0) throw Error(GANMRES_EDEVICE, "getcontext failed");
        t.ctx.uc_stack.ss_sp = t.stack.get();
        t.ctx.uc_stack.ss_size = kStack;
        t.ctx.uc_link = &home;
        const uintptr_t p = reinterpret_cast<uintptr_t>(&t);
        makecontext(&t.ctx, reinterpret_cast<void (*)()>(&coop_entry), 2,
                    static_cast<unsigned>(p & 0xffffffffu), static_cast<unsigned>(p >> 32));
    }
    for (;;) {
        for (auto& tp : tasks)
            if (tp->state == CoopTask::RUN) {
                g_coop = tp.get();
                swapcontext(&home, &tp->ctx);
                g_coop = nullptr;
            }
        int launch = 0, sync = 0, barrier = 0, live = 0;
        for (auto& tp : tasks) {
            launch += tp->state == CoopTask::LAUNCH;
            sync += tp->state == CoopTask::SYNC;
            barrier += tp->state == CoopTask::BARRIER;
            live += tp->state != CoopTask::DONE;
        }
        if (live == 0) break;
        if (launch > 0) {
            // one launch per family (chunks of kMaxGroup classes)
            std::vector<char> taken(n, 0);
            for (int i = 0; i < n; ++i) {
                if (taken[i] || tasks[i]->state != CoopTask::LAUNCH) continue;
                std::vector<int> fam;
                for (int j = i; j < n; ++j)
                    if (!taken[j] && tasks[j]->state == CoopTask::LAUNCH &&
                        tasks[j]->desc.fam == tasks[i]->desc.fam) {
                        fam.push_back(j);
                        taken[j] = 1;
                    }
                for (size_t c0 = 0; c0 < fam.size(); c0 += kMaxGroup) {
                    const int m = static_cast<int>(std::min(fam.size() - c0, size_t(kMaxGroup)));
                    hipError_t rc;
                    if (m == 1) {
                        rc = tasks[fam[c0]]->desc.launch_single(tasks[fam[c0]]->desc, st);
                    } else {
                        const LaunchDesc* ds[kMaxGroup];
                        for (int q = 0; q < m; ++q) ds[q] = &tasks[fam[c0 + q]]->desc;
                        rc = ds[0]->fam->launch_group(ds, m, st);
                    }
                    if (stats) {
                        stats->submitted += m;
                        stats->issued += 1;
                    }
                    for (int q = 0; q < m; ++q) {
                        CoopTask& t = *tasks[fam[c0 + q]];
                        t.state = CoopTask::RUN;
                        if (rc != hipSuccess) {
                            t.fail = 1;
                            t.fail_msg = std::string("kernel launch: ") + hipGetErrorString(rc);
                        }
                    }
                }
            }
            continue;
        }
        if (sync > 0) {
            const hipError_t rc = hipStreamSynchronize(st);
            for (auto& tp : tasks)
                if (tp->state == CoopTask::SYNC) {
                    tp->state = CoopTask::RUN;
                    if (rc != hipSuccess) {
                        tp->fail = 1;
                        tp->fail_msg = std::string("hipStreamSynchronize: ") + hipGetErrorString(rc);
                    }
                }
            continue;
        }
        // every live task waits at a reduction
        long long mx = LLONG_MIN, any = 0;
        for (auto& tp : tasks)
            if (tp->state == CoopTask::BARRIER) {
                if (tp->bop == 0) mx = std::max(mx, tp->bval);
                else any = any || tp->bval != 0;
            }
        for (auto& tp : tasks)
            if (tp->state == CoopTask::BARRIER) {
                tp->bval = tp->bop == 0 ? mx : any;
                tp->state = CoopTask::RUN;
            }
        (void)barrier;
    }
    for (auto& tp : tasks)
        if (tp->err != GANMRES_OK) throw Error(tp->err, tp->err_msg);
}

// Synchronisation points and reductions of code that may run as a task.
static inline void stream_sync(hipStream_t st) {
    if (CoopTask* t = coop_current()) coop_sync(t);
    else HIPCHK(hipStreamSynchronize(st));
}
static inline void event_sync(hipEvent_t ev) {
    // under the scheduler a stream synchronisation covers every event
    if (CoopTask* t = coop_current()) coop_sync(t);
    else HIPCHK(hipEventSynchronize(ev));
}
static inline int group_max(int v) {
    CoopTask* t = coop_current();
    return t ? static_cast<int>(coop_reduce(t, v, 0)) : v;
}
static inline bool group_any(bool v) {
    CoopTask* t = coop_current();
    return t ? coop_reduce(t, v ? 1 : 0, 1) != 0 : v;
}

// ---- small dense FP64 least squares (host) ----------------------------------
// Solve M beta = y (M symmetric positive semi-definite, n <= 65): Cholesky,
// unless it fails or the squared pivot ratio is below 1e-12; then the eigen
// pseudo-inverse with cutoff 1e-12 lambda_max (cyclic Jacobi).
static constexpr double kLsqCutoff = 1e-12;

static bool cholesky_solve(int n, const std::vector<double>& M, const std::vector<double>& y,
                           std::vector<double>& x) {
    std::vector<double> L(n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = M[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return false;
        const double ljj = std::sqrt(d);
        L[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = M[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / ljj;
        }
    }
    double pmin = INFINITY, pmax = 0.0;
    for (int j = 0; j < n; ++j) {
        const double p = L[j * n + j] * L[j * n + j];
        pmin = std::min(pmin, p);
        pmax = std::max(pmax, p);
    }
    if (pmin < kLsqCutoff * pmax) return false;
    std::vector<double> z(n);
    for (int i = 0; i < n; ++i) {
        double s = y[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * z[k];
        z[i] = s / L[i * n + i];
    }
    x.assign(n, 0.0);
    for (int i = n - 1; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
    return true;
}

static void eigen_pinv_solve(int n, const std::vector<double>& M, const std::vector<double>& y,
                             std::vector<double>& x) {
    std::vector<double> A = M, V(n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    double lmax = 0.0;
    for (int i = 0; i < n; ++i) lmax = std::max(lmax, A[i * n + i]);
    x.assign(n, 0.0);
    for (int e = 0; e < n; ++e) {
        const double lam = A[e * n + e];
        if (!(lam > kLsqCutoff * lmax)) continue;
        double proj = 0.0;
        for (int k = 0; k < n; ++k) proj += V[k * n + e] * y[k];
        for (int k = 0; k < n; ++k) x[k] += V[k * n + e] * proj / lam;
    }
}

// beta from the Gram matrix (K x K, row major) of u = [r, g_0, ..., g_{K-2}];
// *fallback (nullable) is set when the pseudo-inverse had to be used.
static std::vector<double> lsq_from_gram(int K, const std::vector<double>& G,
                                         bool* fallback = nullptr) {
    const int n = K - 1;
    const double Grr = G[0];
    std::vector<double> M(n * n), y(n), x;
    for (int i = 0; i < n; ++i) {
        const double Gri = G[i + 1];
        y[i] = -(Grr - Gri);
        for (int j = 0; j < n; ++j) {
            const double Grj = G[j + 1];
            M[i * n + j] = Grr - Gri - Grj + G[(i + 1) * K + (j + 1)];
        }
    }
    const bool chol = cholesky_solve(n, M, y, x);
    if (!chol) eigen_pinv_solve(n, M, y, x);
    if (fallback) *fallback = !chol;
    return x;
}

// ---- the problem -----------------------------------------------------------
class ProblemBase {
   public:
    virtual ~ProblemBase() = default;
    virtual double objective(const void* v, bool keep, double* mismatch) = 0;
    virtual double gradient(const void* v, void* g, bool reuse) = 0;
    virtual double precond(const void* g, void* s) = 0;
    // info: one entry per stacked problem
    virtual void step(const ganmres_solver_params& p, void* v, ganmres_step_info* info) = 0;
    virtual int count() const = 0;
    virtual void deformation(const void* v, void* det, double* stats) = 0;
    virtual void hessian_matvec(const void* v, const void* vt, void* out) = 0;
    virtual void newton_precond(int which, const void* v, const void* r, void* z) = 0;
    virtual void values(double* J, double* mismatch) const = 0;
    virtual void reset() = 0;
    virtual void get_field(int which, int j, void* out) = 0;
    virtual long long workspace_bytes() const = 0;
    // timing
    bool timing = false;
    unsigned tmask = ~0u;  // kernel classes bracketed while timing
    double tms[KC_COUNT] = {};
    long long tcount[KC_COUNT] = {};
    virtual void timing_flush() = 0;
};

template <typename T>
class Problem : public ProblemBase {
   public:
    using CT = C2<T>;
    ganmres_config cfg;
    Dims dm{};
    hipStream_t st;
    int d;
    long long N, NH;
    double h[3], cell, ht;
    double cscale[3];  // h_t / h_c per component
    SpectralPlans<T> plans{};
    SpectralPlans<double> plans64{};  // the FP64 spectrum of v (regulariser)
    std::vector<std::unique_ptr<DevBuf>> bufs;
    DevBuf twbuf[3], twbuf64[3];
    T *m0, *m1, *dX, *dY, *delta, *cfac, *bfac, *b;
    // window tables of dX and dY: the first gather over a new field records
    // its windows (tw() gives that gather table_write = 1), the later ones read them
    int *tabX = nullptr, *tabY = nullptr;
    bool tabX_ok = false, tabY_ok = false;
    static int tw(bool& ok) {
        const int w = ok ? 0 : 1;
        ok = true;
        return w;
    }
    // State / adjoint storage.  Full mode (checkpoint_every == 1): every m^j
    // and lam^j.  Checkpoint mode: m^j at the checkpoint times 0, c, 2c, ...,
    // nt only, c-1 fields for the interior states of a segment (the forward
    // solve passes through them, the backward sweep recomputes into them),
    // and c+1 adjoint fields reused segment by segment.
    bool full = true;
    int cke = 1;
    std::vector<int> bnd;             // checkpoint times
    T* mhist = nullptr;               // full mode: (nt+1) N
    T* lamh = nullptr;                // full mode: (nt+1) N
    std::vector<T*> ck, mint, lpool;  // checkpoint mode
    T* lam_nt = nullptr;
    T* lam0 = nullptr;
    C2<double>* vh[3];
    CT* wh[3];
    CT* sk[3];                   // spectrum of the last search direction (line search)
    // The solver's gradients also yield the next direction's spectrum (in sk,
    // and a copy in ws that its inverse transform consumes): pre_spec_g is
    // the gradient it belongs to, nullptr when none is pending.
    CT* ws[3] = {nullptr, nullptr, nullptr};
    const void* pre_spec_g = nullptr;
    const void* vh_of = nullptr;  // velocity whose spectrum vh holds
    bool reg_from_device = true;  // R(v) of the next finish_J comes from the device sums
    double *partial, *dres;
    // stacked independent 2-D problems (1 for a single problem): per-problem
    // points, regularisation weights and scalars
    int nb = 1;
    long long Nt = 0;
    std::vector<double> alpha_s;
    double* alpha_dev = nullptr;
    double* coef_dev = nullptr;    // combine coefficients, K x nb
    std::vector<double> reg_s;     // R(v) per problem of the last evaluation
    std::vector<double> J_s, mis_s;
    // displacement bounds of the velocity whose departure points are current
    double umax = 0.0;              // >= max |u| (cells per step)
    int ubound = 0, dbound = 0;     // floor-spread bounds for the predictor and for X / Y
    const void* umax_of = nullptr;  // velocity umax belongs to
    hipEvent_t ev_res = nullptr;  // marks a result copy the host waits for while later work runs
    double* hres = nullptr;  // pinned host results
    double* hup = nullptr;   // pinned staging of host -> device tables
    // slots of the device / host result buffers (per-problem values from s)
    static constexpr int kRes = 2048 + kMaxGram * (kMaxGram + 1) / 2 * kMaxSeg;
    static constexpr int R_MIS = 0, R_REG = 256, R_DOT = 512, R_SMAX = 768, R_CROSS = 1024,
                         R_MAX = 1280, R_UMAX = 1536, R_GRAM = 2048;
    long long ws_bytes = 0;
    bool fwd_valid = false;
    const void* fwd_v = nullptr;
    bool adj_valid = false;
    bool y_valid = false;

    // solver
    int wcap = -1;
    std::vector<std::unique_ptr<DevBuf>> ring_v, ring_g;
    std::unique_ptr<DevBuf> qb, gqb, sb;
    std::vector<std::unique_ptr<DevBuf>> aa_r, aa_q;  // GA-AA: (r, q) history
    int aa_cur = 0;
    int acc_cap = -1;
    std::deque<int> hist;
    bool started = false;
    int k = 0;
    std::vector<double> rho_bar, g0inf, Jcur;  // per problem

    // timing events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    std::vector<int> ev_kind;
    std::vector<int> ev_count;  // launches inside each bracketed interval
    size_t ev_used = 0;

    T* alloc_T(long long n) {
        bufs.emplace_back(new DevBuf);
        bufs.back()->alloc(sizeof(T) * (size_t)n);
        ws_bytes += sizeof(T) * n;
        return static_cast<T*>(bufs.back()->p);
    }
    CT* alloc_C(long long n) {
        bufs.emplace_back(new DevBuf);
        bufs.back()->alloc(sizeof(CT) * (size_t)n);
        ws_bytes += sizeof(CT) * n;
        return static_cast<CT*>(bufs.back()->p);
    }

    // count > 1 (2-D only): count problems of shape n stacked along axis 0,
    // with regularisation weights alpha_in[0..count) (nullptr: cfg.alpha)
    Problem(const ganmres_config& c, const void* m0_in, const void* m1_in, hipStream_t s,
            int count = 1, const double* alpha_in = nullptr)
        : cfg(c), st(s) {
        d = c.dim;
        nb = count;
        dm.dim = d;
        dm.n[0] = d == 3 ? c.n[0] : count;
        dm.n[1] = d == 3 ? c.n[1] : c.n[0];
        dm.n[2] = d == 3 ? c.n[2] : c.n[1];
        dm.N = (long long)dm.n[0] * dm.n[1] * dm.n[2];
        dm.n2h = dm.n[2] / 2 + 1;
        dm.NH = (long long)dm.n[0] * dm.n[1] * dm.n2h;
        N = dm.N;
        NH = dm.NH;
        Nt = N / nb;
        alpha_s.assign(nb, c.alpha);
        if (alpha_in)
            for (int i = 0; i < nb; ++i) alpha_s[i] = alpha_in[i];
        reg_s.assign(nb, 0.0);
        J_s.assign(nb, 0.0);
        mis_s.assign(nb, 0.0);
        rho_bar.assign(nb, 1.0);
        g0inf.assign(nb, 0.0);
        Jcur.assign(nb, 0.0);
        cell = 1.0;
        for (int a = 0; a < 3; ++a) {
            h[a] = 2.0 * M_PI / dm.n[a];
            if (a >= 3 - d) cell *= h[a];
        }
        ht = 1.0 / c.nt;
        for (int cc = 0; cc < d; ++cc) cscale[cc] = ht / h[comp_axis(d, cc)];
        // FFT plans and FP64 twiddles
        for (int a = 3 - d; a < 3; ++a) {
            FftPlan<T>& pl = plans.p[a];
            pl.L = dm.n[a];
            pl.nrad = make_radices(pl.L, pl.rad);
            std::vector<CT> tw(pl.L);
            for (int m = 0; m < pl.L; ++m) {
                const double ang = -2.0 * M_PI * m / pl.L;
                tw[m] = cmk(T(std::cos(ang)), T(std::sin(ang)));
            }
            twbuf[a].alloc(sizeof(CT) * pl.L);
            HIPCHK(hipMemcpyAsync(twbuf[a].p, tw.data(), sizeof(CT) * pl.L, hipMemcpyHostToDevice, st));
            pl.tw = static_cast<const CT*>(twbuf[a].p);
            FftPlan<double>& p64 = plans64.p[a];
            p64.L = pl.L;
            p64.nrad = pl.nrad;
            for (int r = 0; r < kMaxRadices; ++r) p64.rad[r] = pl.rad[r];
            std::vector<C2<double>> tw64(pl.L);
            for (int m = 0; m < pl.L; ++m) {
                const double ang = -2.0 * M_PI * m / pl.L;
                tw64[m] = cmk(std::cos(ang), std::sin(ang));
            }
            twbuf64[a].alloc(sizeof(C2<double>) * pl.L);
            HIPCHK(hipMemcpyAsync(twbuf64[a].p, tw64.data(), sizeof(C2<double>) * pl.L,
                                  hipMemcpyHostToDevice, st));
            p64.tw = static_cast<const C2<double>*>(twbuf64[a].p);
        }
        const int nt = c.nt;
        m0 = alloc_T(N);
        m1 = alloc_T(N);
        cke = c.checkpoint_every;
        full = cke == 1;
        for (int j = 0; j < nt; j += cke) bnd.push_back(j);
        bnd.push_back(nt);
        if (full) {
            mhist = alloc_T((nt + 1) * N);
            lamh = alloc_T((nt + 1) * N);
            lam_nt = lamh + (long long)nt * N;
            lam0 = lamh;
        } else {
            for (size_t i = 0; i < bnd.size(); ++i) ck.push_back(alloc_T(N));
            for (int i = 0; i < std::min(cke, nt) - 1; ++i) mint.push_back(alloc_T(N));
            for (int i = 0; i < std::min(cke, nt) + 1; ++i) lpool.push_back(alloc_T(N));
            lam_nt = lpool[0];
        }
        dX = alloc_T(d * N);
        dY = alloc_T(d * N);
        for (int** tab : {&tabX, &tabY}) {
            const long long ints = window_table_ints<T>(dm);
            bufs.emplace_back(new DevBuf);
            bufs.back()->alloc(sizeof(int) * (size_t)ints);
            ws_bytes += sizeof(int) * ints;
            *tab = static_cast<int*>(bufs.back()->p);
        }
        const bool compressible = !c.incompressible;
        delta = compressible ? alloc_T(N) : nullptr;
        cfac = (compressible && c.model == GANMRES_CONTINUITY) ? alloc_T(N) : nullptr;
        bfac = (compressible && c.model == GANMRES_ADVECTION) ? alloc_T(N) : nullptr;
        b = alloc_T(d * N);
        for (int cc = 0; cc < 3; ++cc) {
            vh[cc] = nullptr;
            if (cc < d) {
                bufs.emplace_back(new DevBuf);
                bufs.back()->alloc(sizeof(C2<double>) * (size_t)NH);
                ws_bytes += sizeof(C2<double>) * NH;
                vh[cc] = static_cast<C2<double>*>(bufs.back()->p);
            }
            wh[cc] = cc < d ? alloc_C(NH) : nullptr;
            sk[cc] = cc < d ? alloc_C(NH) : nullptr;
        }
        {
            bufs.emplace_back(new DevBuf);
            bufs.back()->alloc(sizeof(double) * kGramPartialDoubles);
            partial = static_cast<double*>(bufs.back()->p);
            bufs.emplace_back(new DevBuf);
            bufs.back()->alloc(sizeof(double) * kMaxSeg);
            alpha_dev = static_cast<double*>(bufs.back()->p);
            bufs.emplace_back(new DevBuf);
            bufs.back()->alloc(sizeof(double) * (GANMRES_MAX_WINDOW + 1) * kMaxSeg);
            coef_dev = static_cast<double*>(bufs.back()->p);
        }
        // the reductions write their results straight into this pinned,
        // mapped host buffer (dres is its device address): a result is on the
        // host once the stream has passed its reduction, with no copy
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hres), sizeof(double) * kRes,
                             hipHostMallocMapped | hipHostMallocCoherent));
        HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&dres), hres, 0));
        HIPCHK(hipEventCreateWithFlags(&ev_res, hipEventDisableTiming));
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hup), sizeof(double) * (GANMRES_MAX_WINDOW + 1) * kMaxSeg,
                             hipHostMallocDefault));
        for (int i = 0; i < nb; ++i) hup[i] = alpha_s[i];
        HIPCHK(hipMemcpyAsync(alpha_dev, hup, sizeof(double) * nb, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(m0, m0_in, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(m1, m1_in, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(mstate(0), m0_in, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        autotune_tile();
    }

    // ---- 2-D gather tile autotuner ------------------------------------------
    // The tile height of the 2-D semi-Lagrangian kernels (points per thread 8,
    // 4 or 2: tiles of 64 x 32, 64 x 16 or 64 x 8 points) is chosen per grid
    // (stacked count and size) and element type by timing the gather step of
    // each variant on this problem's template image with zero displacement
    // (window tables recorded first, as in a solve), and remembered for the
    // process.  Small grids gain workgroups from short tiles; large ones keep
    // the staging of fewer, taller windows.  Every variant gives the same
    // values: only the work partition changes.
    int tile_choice = 0;
    double tile_us[3] = {0.0, 0.0, 0.0};  // per launch, variants 8, 4, 2
    void autotune_tile() {
        if (d != 2) return;
        static std::mutex mu;
        static std::map<std::tuple<int, int, int, int>, std::pair<int, std::vector<double>>> cache;
        const auto key = std::make_tuple(dm.n[0], dm.n[1], dm.n[2], (int)sizeof(T));
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = cache.find(key);
            if (it != cache.end()) {
                dm.tile = tile_choice = it->second.first;
                for (int i = 0; i < 3; ++i) tile_us[i] = it->second.second[i];
                return;
            }
        }
        constexpr int kReps = 5;
        const int variants[3] = {8, 4, 2};
        HIPCHK(hipMemsetAsync(dX, 0, sizeof(T) * d * N, st));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        int best = kTile2Default;
        double best_us = INFINITY;
        for (int i = 0; i < 3; ++i) {
            dm.tile = variants[i];
            HIPCHK(launch_sl_step<T>(dm, m0, dX, nullptr, 0, b, st, tabX, 1));
            HIPCHK(launch_sl_step<T>(dm, m0, dX, nullptr, 0, b, st, tabX, 0));
            HIPCHK(hipEventRecord(e0, st));
            for (int r = 0; r < kReps; ++r) HIPCHK(launch_sl_step<T>(dm, m0, dX, nullptr, 0, b, st, tabX, 0));
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            tile_us[i] = 1e3 * ms / kReps;
            if (tile_us[i] < best_us) {
                best_us = tile_us[i];
                best = variants[i];
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        dm.tile = tile_choice = best;
        tabX_ok = false;
        std::lock_guard<std::mutex> lk(mu);
        cache[key] = {best, std::vector<double>(tile_us, tile_us + 3)};
    }

    ~Problem() override {
        if (ev_res) (void)hipEventDestroy(ev_res);
        if (hres) (void)hipHostFree(hres);
        if (hup) (void)hipHostFree(hup);
        for (auto& e : ev_pool) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }

    long long workspace_bytes() const override {
        long long s = ws_bytes;
        for (auto& r : ring_v) s += r->bytes;
        for (auto& r : ring_g) s += r->bytes;
        for (auto& r : aa_r) s += r->bytes;
        for (auto& r : aa_q) s += r->bytes;
        if (qb) s += qb->bytes + gqb->bytes + sb->bytes;
        if (coarse) s += coarse->workspace_bytes();  // the two-level preconditioner's grid
        return s;
    }

    // -- timing -------------------------------------------------------------
    // Only the selected classes are bracketed: every event pair costs the
    // stream some microseconds, so a run that times one class leaves the
    // others undisturbed.  The events skip the system-scope fence (the
    // timestamps need no host-visible memory ordering).
    bool tcur = false;
    void tbegin(int kind) {
        tcur = timing && ((tmask >> kind) & 1u);
        if (!tcur) return;
        if (ev_used == ev_pool.size()) {
            hipEvent_t a, b2;
            HIPCHK(hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
            HIPCHK(hipEventCreateWithFlags(&b2, hipEventDisableSystemFence));
            ev_pool.push_back({a, b2});
            ev_kind.push_back(kind);
            ev_count.push_back(1);
        }
        ev_kind[ev_used] = kind;
        HIPCHK(hipEventRecord(ev_pool[ev_used].first, st));
    }
    void tend(int launches = 1) {
        if (!tcur) return;
        tcur = false;
        ev_count[ev_used] = launches;
        HIPCHK(hipEventRecord(ev_pool[ev_used].second, st));
        ++ev_used;
        if (ev_used >= 4096) timing_flush();
    }
    void timing_flush() override {
        if (ev_used == 0) return;
        HIPCHK(hipStreamSynchronize(st));
        for (size_t i = 0; i < ev_used; ++i) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev_pool[i].first, ev_pool[i].second));
            tms[ev_kind[i]] += ms;
            tcount[ev_kind[i]] += ev_count[i];
        }
        ev_used = 0;
    }

    template <typename F>
    void run(int kind, F&& f) {
        tbegin(kind);
        HIPCHK(f());
        tend();
    }
    // n launches of one class back to back (f(i) enqueues the i-th and nothing
    // else): one pair of timing events brackets them all, since every event in
    // the stream pauses the device briefly
    template <typename F>
    void run_seq(int kind, int n, F&& f) {
        if (n <= 0) return;
        tbegin(kind);
        for (int i = 0; i < n; ++i) HIPCHK(f(i));
        tend(n);
    }

    // result slots [at, at + n) on the host (synchronises).  Every slot is
    // written by the reductions in stream order: the host reads a slot only
    // after a synchronisation that follows its reduction, and before it
    // launches another reduction into the same slot.
    const double* fetch(int at, int n) {
        (void)n;
        stream_sync(st);
        return hres + at;
    }
    // scalar and velocity fields as segments (one per stacked problem)
    Seg sseg() const { return Seg{nb, 1, Nt, N}; }
    Seg vseg() const { return Seg{nb, d, Nt, N}; }

    const T* comp(const void* v, int c) const { return static_cast<const T*>(v) + c * N; }
    T* comp(void* v, int c) const { return static_cast<T*>(v) + c * N; }

    SpecOpParams specop(bool leray) const {
        SpecOpParams s;
        s.dim = d;
        s.p = cfg.reg_order;
        s.alpha = cfg.alpha;
        s.leray = leray ? 1 : 0;
        s.alpha_seg = nb > 1 ? alpha_dev : nullptr;
        return s;
    }

    // -- per-velocity preparation ---------------------------------------------
    // v^, R(v) (device sums per problem -> reg_s), divergence, departure points and
    // stationary source factors.
    void spectrum_of(const void* v) {
        const T* vin[3] = {comp(v, 0), comp(v, 1), d == 3 ? comp(v, 2) : nullptr};
        run(KC_RFFT, [&] { return launch_rfft<T, double>(dm, plans64, vin, vh, d, st); });
        run(KC_REDUCE, [&] {
            return launch_spec_regvalue<double>(dm, specop(false), vh, partial, dres + R_REG, st);
        });
        vh_of = v;
        reg_from_device = true;
    }

    void set_bounds(const void* v, double um) {
        umax = um;
        umax_of = v;
        // the classes of a group handle take the largest bound, so that they
        // select the same kernel variants and their launches merge
        ubound = group_max(spread_bound(um * (1.0 + 1e-6)));
        dbound = group_max(displacement_bound(um, d));
    }

    // max |u| of a velocity over all problems (reduction + sync)
    double velocity_max(const void* v) {
        run(KC_REDUCE, [&] {
            return launch_velocity_max<T>(dm, static_cast<const T*>(v), cscale, partial,
                                          dres + R_UMAX, st);
        });
        return fetch(R_UMAX, 1)[0];
    }

    // trial = true: a line-search trial whose R(v) the caller supplies and
    // whose spectrum is not needed (vh keeps the current iterate's); umax_known
    // >= 0 is a known bound on max |u| of v (else it is reduced on the device)
    void prepare(const void* v, bool needY, bool trial = false, double umax_known = -1.0) {
        if (umax_known >= 0.0) {
            if (!trial) spectrum_of(v);
            set_bounds(v, umax_known);
        } else {
            // the bound picks the gather variants: reduce it first and let the
            // spectrum of v run while the host waits for it
            run(KC_REDUCE, [&] {
                return launch_velocity_max<T>(dm, static_cast<const T*>(v), cscale, partial,
                                              dres + R_UMAX, st);
            });
            HIPCHK(hipEventRecord(ev_res, st));
            if (!trial) spectrum_of(v);
            event_sync(ev_res);
            set_bounds(v, hres[R_UMAX]);
        }
        if (delta) {
            const double one = 1.0;
            for (int cc = 0; cc < d; ++cc) {
                const T* f = comp(v, cc);
                run(KC_DERIV, [&] {
                    return launch_deriv_axis<T>(dm, plans, comp_axis(d, cc), &f, nullptr, &one, 1,
                                                cc > 0, delta, st);
                });
            }
        }
        run(KC_CHAR, [&] {
            return launch_characteristics<T>(dm, static_cast<const T*>(v), cscale, ubound, dX,
                                             needY ? dY : nullptr, st);
        });
        tabX_ok = false;
        if (needY) tabY_ok = false;
        y_valid = needY;
        if (cfac)
            run(KC_FACTOR, [&] {
                return launch_source_factor<T>(dm, delta, dX, ht, -1.0, dbound, cfac, st, tabX, tw(tabX_ok));
            });
        if (bfac && needY)
            run(KC_FACTOR, [&] {
                return launch_source_factor<T>(dm, delta, dY, ht, +1.0, dbound, bfac, st, tabY, tw(tabY_ok));
            });
    }

    void ensure_Y(const void* v) {
        if (y_valid) return;
        // characteristics for -v only; the bounds of v are still current
        run(KC_CHAR, [&] {
            return launch_characteristics<T>(dm, static_cast<const T*>(v), cscale, ubound, nullptr,
                                             dY, st);
        });
        tabY_ok = false;
        if (bfac)
            run(KC_FACTOR, [&] {
                return launch_source_factor<T>(dm, delta, dY, ht, +1.0, dbound, bfac, st, tabY, tw(tabY_ok));
            });
        y_valid = true;
    }

    // where the forward solve keeps m^j
    int ck_index(int j) const {
        for (size_t i = 0; i < bnd.size(); ++i)
            if (bnd[i] == j) return (int)i;
        return -1;
    }
    T* mstate(int j) {
        if (full) return mhist + (long long)j * N;
        const int i = ck_index(j);
        // interior states: consecutive ones land in different buffers when c > 2,
        // and with c = 2 no two interior states are consecutive
        return i >= 0 ? ck[i] : mint[j % (int)mint.size()];
    }

    void forward() {
        run_seq(KC_SL, cfg.nt, [&](int j) {
            return launch_sl_step<T>(dm, mstate(j), dX, cfac, dbound, mstate(j + 1), st, tabX, tw(tabX_ok));
        });
    }

    // mismatch sums per problem -> dres[R_MIS..]; optionally lam^nt = m1 - m^nt
    void mismatch(bool write_lam) {
        run(KC_REDUCE, [&] {
            return launch_sumsq_diff<T>(mstate(cfg.nt), m1, write_lam ? lam_nt : nullptr, sseg(),
                                        partial, dres + R_MIS, st);
        });
    }

    // J per problem (J_s, mis_s) and their sum
    double finish_J(double* mis_out) {
        stream_sync(st);
        return J_from_host(mis_out);
    }
    // the ingredients of J reach the host behind an event (see J_from_host);
    // until it is taken up, no reduction into their slots is launched
    void J_to_host() {
        J_pending = false;
        HIPCHK(hipEventRecord(ev_res, st));
    }
    double J_from_host(double* mis_out) {
        double Jt = 0.0, mt = 0.0;
        for (int i = 0; i < nb; ++i) {
            mis_s[i] = 0.5 * cell * hres[R_MIS + i];
            if (reg_from_device) reg_s[i] = cell / double(Nt) * hres[R_REG + i];
            J_s[i] = mis_s[i] + 0.5 * alpha_s[i] * reg_s[i];
            Jt += J_s[i];
            mt += mis_s[i];
        }
        reg_from_device = false;
        if (mis_out) *mis_out = mt;
        return Jt;
    }

    // J at a line-search trial v with known regulariser values R (per problem)
    double objective_trial(const void* v, const std::vector<double>& R, double um) {
        prepare(v, false, true, um);
        forward();
        mismatch(false);
        fwd_valid = true;
        fwd_v = v;
        adj_valid = false;
        reg_s = R;
        reg_from_device = false;
        return finish_J(nullptr);
    }

    double objective(const void* v, bool keep, double* mis) override {
        pre_g = nullptr;
        pre_spec_g = nullptr;
        prepare(v, false);
        forward();
        mismatch(false);
        fwd_valid = keep;
        fwd_v = keep ? v : nullptr;
        adj_valid = false;
        return finish_J(mis);
    }

    double trap_weight(int t) const {
        const double w = (t == 0 || t == cfg.nt) ? 0.5 * ht : ht;
        return cfg.model == GANMRES_CONTINUITY ? -w : w;
    }

    // body force over the given time levels: advection b += w lam grad m,
    // continuity b -= w pi grad lam (one launch per axis)
    void body_force(const std::vector<const T*>& m, const std::vector<const T*>& lam,
                    const std::vector<double>& w, bool accumulate) {
        const bool cont = cfg.model == GANMRES_CONTINUITY;
        for (int cc = 0; cc < d; ++cc)
            run(KC_DERIV, [&] {
                return launch_deriv_axis<T>(dm, plans, comp_axis(d, cc), cont ? lam.data() : m.data(),
                                            cont ? m.data() : lam.data(), w.data(), (int)w.size(),
                                            accumulate ? 1 : 0, comp(b, cc), st);
            });
    }

    // adjoint backward in time and the body force b (lam^nt already written)
    void backward() {
        const int nt = cfg.nt;
        if (full) {
            run_seq(KC_SL, nt, [&](int i) {
                const int j = nt - 1 - i;
                return launch_sl_step<T>(dm, lamh + (long long)(j + 1) * N, dY, bfac, dbound,
                                         lamh + (long long)j * N, st, tabY, tw(tabY_ok));
            });
            std::vector<const T*> mp(nt + 1), lp(nt + 1);
            std::vector<double> w(nt + 1);
            for (int t = 0; t <= nt; ++t) {
                mp[t] = mhist + (long long)t * N;
                lp[t] = lamh + (long long)t * N;
                w[t] = trap_weight(t);
            }
            body_force(mp, lp, w, false);
            adj_valid = true;
            return;
        }
        // checkpoint mode: segments [bnd[s], bnd[s+1]] from the last to the first
        const int nseg = (int)bnd.size() - 1;
        int top = 0;  // lpool index holding lam at the segment's end time
        for (int sgi = nseg - 1; sgi >= 0; --sgi) {
            const int j0 = bnd[sgi], j1 = bnd[sgi + 1], len = j1 - j0;
            std::vector<T*> mp(len + 1), lp(len + 1);
            mp[0] = ck[sgi];
            mp[len] = ck[sgi + 1];
            for (int i = 1; i < len; ++i) mp[i] = mint[i - 1];
            run_seq(KC_SL, len - 1, [&](int q) {
                const int i = q + 1;
                return launch_sl_step<T>(dm, mp[i - 1], dX, cfac, dbound, mp[i], st, tabX, tw(tabX_ok));
            });
            std::vector<int> idx;
            for (int i = 0; i < (int)lpool.size(); ++i)
                if (i != top) idx.push_back(i);
            lp[len] = lpool[top];
            int newtop = top;
            for (int i = len - 1, q = 0; i >= 0; --i, ++q) {
                lp[i] = lpool[idx[q]];
                if (i == 0) newtop = idx[q];
            }
            run_seq(KC_SL, len, [&](int q) {
                const int i = len - 1 - q;
                return launch_sl_step<T>(dm, lp[i + 1], dY, bfac, dbound, lp[i], st, tabY, tw(tabY_ok));
            });
            // time level j0 belongs to the previous segment, except t = 0
            const int i0 = sgi == 0 ? 0 : 1;
            std::vector<const T*> fm, fl;
            std::vector<double> w;
            for (int i = i0; i <= len; ++i) {
                fm.push_back(mp[i]);
                fl.push_back(lp[i]);
                w.push_back(trap_weight(j0 + i));
            }
            body_force(fm, fl, w, sgi != nseg - 1);
            top = newtop;
            if (sgi == 0) lam0 = lp[0];
        }
        adj_valid = true;
    }

    double gradient(const void* v, void* g, bool reuse) override {
        pre_g = nullptr;
        pre_spec_g = nullptr;
        gradient_async(v, g, reuse, true);
        return resolve_J();
    }

    // The gradient without waiting for J: J reaches the host behind ev_res and
    // resolve_J() (or any later synchronisation followed by resolve_J) takes it
    // up.  The solver calls this where J is already known (the accepted trial's
    // forward solve is reused) or is needed only at the end of the step.
    bool J_pending = false;
    bool J_event = false;  // an event follows the mismatch (else: wait for the stream)
    double resolve_J() {
        if (!J_pending) return 0.0;
        if (J_event) event_sync(ev_res);
        else stream_sync(st);
        J_pending = false;
        return J_from_host(nullptr);
    }
    // J_event: record an event behind the mismatch, so that resolve_J waits
    // for it alone (an event in the stream costs the device a short pause;
    // the solver, which takes J up after a later synchronisation, records none)
    // want_pre: the assembly also leaves the spectrum of the preconditioned
    // direction of g (for the precond_launch of the same g that follows)
    void gradient_async(const void* v, void* g, bool reuse, bool J_event_ = false,
                        bool want_pre = false) {
        if (reuse) {
            if (!fwd_valid || fwd_v != v)
                throw Error(GANMRES_ESTATE, "reuse_forward without a kept forward solve for this v");
            ensure_Y(v);
        } else {
            prepare(v, true);
            forward();
            fwd_valid = true;
            fwd_v = v;
        }
        mismatch(true);
        // J reaches the host while the adjoint and the assembly run
        J_event = J_event_;
        if (J_event) J_to_host();
        backward();
        // assembly g = alpha L v + [P] b (the operator fused with the last
        // forward and the first inverse pass)
        const T* bin[3] = {comp(b, 0), comp(b, 1), d == 3 ? comp(b, 2) : nullptr};
        run(KC_RFFT, [&] { return launch_rfft<T, T>(dm, plans, bin, wh, d, st, 1); });
        if (want_pre && !ws[0])
            for (int cc = 0; cc < d; ++cc) ws[cc] = alloc_C(NH);
        run(KC_SPEC, [&] {
            return launch_spec_fused<T>(dm, plans, kSpecGrad, specop(cfg.incompressible != 0), wh, vh,
                                        want_pre ? sk : nullptr, st, want_pre ? ws : nullptr);
        });
        pre_spec_g = want_pre ? g : nullptr;
        T* gout[3] = {comp(g, 0), comp(g, 1), d == 3 ? comp(g, 2) : nullptr};
        run(KC_IRFFT, [&] { return launch_irfft<T>(dm, plans, wh, gout, nullptr, 1.0 / Nt, d, st, 1); });
        J_pending = true;
    }

    double precond(const void* g, void* s) override {
        pre_g = nullptr;
        pre_spec_g = nullptr;
        precond_keep(g, s, false);
        double t = 0.0;
        for (int i = 0; i < nb; ++i) t += gs_s[i];
        return t;
    }

    // s = -(alpha L)^-1 g; gs_s = <g, s>_h per problem; keep: also keep s^,
    // max |s| (cells per step) and the regulariser cross terms of the line
    // v + rho s (dres[R_CROSS..], see launch_spec_cross)
    void precond_keep(const void* g, void* s, bool keep) {
        precond_launch(g, s, keep);
        stream_sync(st);
        precond_collect(keep);
    }
    // the launches of precond_keep and the copy of its results to the host
    void precond_launch(const void* g, void* s, bool keep) {
        T* sout[3] = {comp(s, 0), comp(s, 1), d == 3 ? comp(s, 2) : nullptr};
        if (keep && pre_spec_g == g) {
            // the direction's spectrum came with the gradient's assembly: only
            // its inverse transform and the scalars remain
            pre_spec_g = nullptr;
            run(KC_REDUCE, [&] {
                return launch_spec_cross<T>(dm, specop(false), vh, sk, partial, dres + R_CROSS, st);
            });
            run(KC_IRFFT, [&] { return launch_irfft<T>(dm, plans, ws, sout, nullptr, 1.0 / Nt, d, st, 0); });
            run(KC_REDUCE, [&] {
                return launch_dot<T>(static_cast<const T*>(g), static_cast<const T*>(s), vseg(), partial,
                                     dres + R_DOT, st);
            });
            run(KC_REDUCE, [&] {
                return launch_velocity_max<T>(dm, static_cast<const T*>(s), cscale, partial,
                                              dres + R_SMAX, st);
            });
            return;
        }
        pre_spec_g = nullptr;
        const T* gin[3] = {comp(g, 0), comp(g, 1), d == 3 ? comp(g, 2) : nullptr};
        run(KC_RFFT, [&] { return launch_rfft<T, T>(dm, plans, gin, wh, d, st, 1); });
        run(KC_SPEC, [&] {
            return launch_spec_fused<T>(dm, plans, kSpecPrecond, specop(cfg.incompressible != 0), wh,
                                        nullptr, keep ? sk : nullptr, st);
        });
        if (keep)
            run(KC_REDUCE, [&] {
                return launch_spec_cross<T>(dm, specop(false), vh, sk, partial, dres + R_CROSS, st);
            });
        run(KC_IRFFT, [&] { return launch_irfft<T>(dm, plans, wh, sout, nullptr, 1.0 / Nt, d, st, 1); });
        run(KC_REDUCE, [&] {
            return launch_dot<T>(static_cast<const T*>(g), static_cast<const T*>(s), vseg(), partial,
                                 dres + R_DOT, st);
        });
        if (keep)
            run(KC_REDUCE, [&] {
                return launch_velocity_max<T>(dm, static_cast<const T*>(s), cscale, partial,
                                              dres + R_SMAX, st);
            });
    }
    // after the stream has synchronised: the results of precond_launch
    void precond_collect(bool keep) {
        if (keep) {
            smax = hres[R_SMAX];
            crossA.assign(hres + R_CROSS, hres + R_CROSS + nb);
            crossB.assign(hres + R_CROSS + nb, hres + R_CROSS + 2 * nb);
        }
        gs_s.resize(nb);
        for (int i = 0; i < nb; ++i) gs_s[i] = cell * hres[R_DOT + i];
    }
    double smax = 0.0;          // max |u| of the last kept search direction
    std::vector<double> gs_s;   // <g, s>_h per problem of the last preconditioning
    std::vector<double> crossA, crossB;  // regulariser cross sums of the kept direction
    // The direction of the next iteration, launched at the end of a solver
    // step so that its results reach the host with the step's own
    // synchronisation: the gradient it belongs to (nullptr: none pending).
    // Any other use of the handle forgets it.
    const void* pre_g = nullptr;

    // max |a| per problem
    std::vector<double> maxabs(const T* a) {
        run(KC_REDUCE, [&] { return launch_maxabs<T>(a, vseg(), partial, dres + R_MAX, st); });
        const double* r = fetch(R_MAX, nb);
        return std::vector<double>(r, r + nb);
    }

    void get_field(int which, int j, void* out) override {
        if (j < 0 || j > cfg.nt || (which != 0 && which != 1))
            throw Error(GANMRES_EINVAL, "field index out of range");
        if (which == 1 && !adj_valid) throw Error(GANMRES_ESTATE, "no adjoint solve available");
        const T* src = nullptr;
        if (which == 0) {
            src = full ? mhist + (long long)j * N : (ck_index(j) >= 0 ? ck[ck_index(j)] : nullptr);
            if (!src) throw Error(GANMRES_ESTATE, "state not kept (not a checkpoint time)");
        } else {
            src = full ? lamh + (long long)j * N : (j == 0 ? lam0 : nullptr);
            if (!src) throw Error(GANMRES_ESTATE, "adjoint not kept at this time (checkpoint mode)");
        }
        HIPCHK(hipMemcpyAsync(out, src, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
        stream_sync(st);
    }

    // ---- Gauss-Newton-Krylov baseline (Appendix A) ---------------------------
    // Gauss-Newton Hessian matvec H_gn[v] vt = alpha L vt + [P] int lt grad m dt
    // (eqs. e:hessian-matvec, e:incremental-state, e:incremental-adjoint, the
    // terms carrying lam dropped): the incremental state is integrated along
    // the state's characteristics with the trapezoidal rule for its source
    // f = -vt . grad m, the Gauss-Newton adjoint with the adjoint's scheme and
    // final value -mt(1).  With g^j = mt^j + h_t/2 f^j the state step is one
    // gather, g^{j+1} = I[g^j](X) + h_t f^{j+1}; the adjoint is carried as
    // L^j = -lt^j (linear), so the body force takes the weights -w_j.
    std::vector<std::unique_ptr<DevBuf>> nk_bufs;  // sources (nt+1) N, g ping-pong 2 N
    C2<double>* vth[3] = {nullptr, nullptr, nullptr};
    void ensure_matvec_buffers() {
        if (!nk_bufs.empty()) return;
        auto add = [&](size_t bytes) {
            nk_bufs.emplace_back(new DevBuf);
            nk_bufs.back()->alloc(bytes);
            ws_bytes += (long long)bytes;
            return nk_bufs.back()->p;
        };
        add(sizeof(T) * (cfg.nt + 1) * N);
        for (int i = 0; i < 2; ++i) add(sizeof(T) * N);
        for (int c = 0; c < d; ++c) vth[c] = static_cast<C2<double>*>(add(sizeof(C2<double>) * NH));
    }

    void check_newton_setup() const {
        if (cfg.model != GANMRES_ADVECTION || !full || nb != 1)
            throw Error(GANMRES_EINVAL,
                        "the Gauss-Newton Hessian needs the advection model, the full state history "
                        "(checkpoint_every = 1) and a single problem");
    }

    // the caller's v may have changed since any earlier call: solve the state again
    void hessian_matvec(const void* v, const void* vt, void* out) override {
        pre_g = nullptr;
        pre_spec_g = nullptr;
        check_newton_setup();
        prepare(v, true);
        forward();
        fwd_valid = true;
        fwd_v = v;
        gn_matvec(v, vt, out);
    }

    // H_gn[v] vt with the state history, departure points and adjoint factors of
    // v current
    void gn_matvec(const void* v, const void* vt, void* out, bool data_only = false) {
        ensure_matvec_buffers();
        ensure_Y(v);
        adj_valid = false;  // lamh is about to hold the incremental adjoint
        const int nt = cfg.nt;
        T* f = static_cast<T*>(nk_bufs[0]->p);  // h_t f^j = -h_t vt . grad m^j
        T* ga = static_cast<T*>(nk_bufs[1]->p);
        T* gb = static_cast<T*>(nk_bufs[2]->p);
        const double wsrc = -ht;
        for (int j = 0; j <= nt; ++j) {
            const T* mj = mstate(j);
            for (int c = 0; c < d; ++c) {
                const T* vc = comp(vt, c);
                run(KC_DERIV, [&] {
                    return launch_deriv_axis<T>(dm, plans, comp_axis(d, c), &mj, &vc, &wsrc, 1,
                                                c > 0, f + (long long)j * N, st);
                });
            }
        }
        const std::vector<double> mhalf(1, -0.5);
        // g^0 = h_t f^0 / 2
        run(KC_VEC, [&] { return launch_axpy<T>(f, mhalf.data(), f, ga, sseg(), st); });
        for (int j = 0; j < nt; ++j) {
            run(KC_SL, [&] {
                return launch_sl_step_add<T>(dm, ga, dX, f + (long long)(j + 1) * N, dbound, gb, st, tabX, tw(tabX_ok));
            });
            std::swap(ga, gb);
        }
        // L^nt = mt^nt = g^nt - h_t f^nt / 2, then L^j = [c_b] I[L^{j+1}](Y)
        run(KC_VEC, [&] {
            return launch_axpy<T>(ga, mhalf.data(), f + (long long)nt * N, lamh + (long long)nt * N,
                                  sseg(), st);
        });
        for (int j = nt - 1; j >= 0; --j)
            run(KC_SL, [&] {
                return launch_sl_step<T>(dm, lamh + (long long)(j + 1) * N, dY, bfac, dbound,
                                         lamh + (long long)j * N, st, tabY, tw(tabY_ok));
            });
        std::vector<const T*> mp(nt + 1), lp(nt + 1);
        std::vector<double> w(nt + 1);
        for (int t = 0; t <= nt; ++t) {
            mp[t] = mhist + (long long)t * N;
            lp[t] = lamh + (long long)t * N;
            w[t] = -trap_weight(t);
        }
        body_force(mp, lp, w, false);
        // assembly: alpha L vt + [P] b (FP64 spectrum of vt, as for v); data_only:
        // [P] b alone (the data term of the two-level preconditioner)
        const T* bin[3] = {comp(b, 0), comp(b, 1), d == 3 ? comp(b, 2) : nullptr};
        T* hout[3] = {comp(out, 0), comp(out, 1), d == 3 ? comp(out, 2) : nullptr};
        if (data_only) {
            run(KC_RFFT, [&] { return launch_rfft<T, T>(dm, plans, bin, wh, d, st); });
            run(KC_SPEC, [&] {
                return launch_spec_pow<T>(dm, specop(cfg.incompressible != 0), wh, wh, 0.0, 1.0, 0, st);
            });
            run(KC_IRFFT, [&] { return launch_irfft<T>(dm, plans, wh, hout, nullptr, 1.0 / Nt, d, st); });
        } else {
            const T* vin[3] = {comp(vt, 0), comp(vt, 1), d == 3 ? comp(vt, 2) : nullptr};
            run(KC_RFFT, [&] { return launch_rfft<T, double>(dm, plans64, vin, vth, d, st); });
            run(KC_RFFT, [&] { return launch_rfft<T, T>(dm, plans, bin, wh, d, st, 1); });
            run(KC_SPEC, [&] {
                return launch_spec_fused<T>(dm, plans, kSpecGrad, specop(cfg.incompressible != 0), wh,
                                            vth, nullptr, st);
            });
            run(KC_IRFFT, [&] { return launch_irfft<T>(dm, plans, wh, hout, nullptr, 1.0 / Nt, d, st, 1); });
        }
    }

    // ---- preconditioners of the Newton step (Appendix A) ---------------------
    // M^-1 r for "h0rpc" (GMRES on the zero-velocity Hessian in its left
    // regularisation-preconditioned form) and "2lrpcsym" (CG on the
    // symmetric regularisation-preconditioned Hessian of the problem on the
    // grid with half the cells, high frequencies by (alpha L)^-1).  Both inner
    // solves stop at a relative residual of kPcTol or after kPcMaxit
    // iterations.  The callers hold q = -r, the negated PCG residual.
    static constexpr int kPcMaxit = 10;
    static constexpr double kPcTol = 1e-1;
    std::vector<std::unique_ptr<DevBuf>> pc_bufs;
    T* pc_alloc(long long elems) {
        pc_bufs.emplace_back(new DevBuf);
        pc_bufs.back()->alloc(sizeof(T) * (size_t)elems);
        ws_bytes += sizeof(T) * elems;
        return static_cast<T*>(pc_bufs.back()->p);
    }
    T* gm0 = nullptr;                 // grad m0
    T* pcv[kPcMaxit + 1] = {};        // Arnoldi basis
    T* pcw = nullptr;                 // GMRES work vector
    T* pcx = nullptr;                 // pointwise data term
    T* qold = nullptr;                // previous -r of the flexible PCG

    void ensure_h0() {
        if (gm0) return;
        ensure_matvec_buffers();
        gm0 = pc_alloc(d * N);
        const double one = 1.0;
        for (int c = 0; c < d; ++c) {
            const T* f = m0;
            run(KC_DERIV, [&] {
                return launch_deriv_axis<T>(dm, plans, comp_axis(d, c), &f, nullptr, &one, 1, 0,
                                            gm0 + (long long)c * N, st);
            });
        }
        for (int i = 0; i <= kPcMaxit; ++i) pcv[i] = pc_alloc(d * N);
        pcw = pc_alloc(d * N);
        pcx = pc_alloc(d * N);
    }

    // out = (alpha L)^-1 [P] H0 x, H0 x = alpha L x + [P] grad m0 (grad m0 . x)
    void h0_left(const T* x, T* out) {
        run(KC_VEC, [&] { return launch_outer<T>(gm0, x, pcx, d, N, st); });
        const T* xin[3] = {comp(x, 0), comp(x, 1), d == 3 ? comp(x, 2) : nullptr};
        run(KC_RFFT, [&] { return launch_rfft<T, double>(dm, plans64, xin, vth, d, st); });
        const T* gin[3] = {comp(pcx, 0), comp(pcx, 1), d == 3 ? comp(pcx, 2) : nullptr};
        run(KC_RFFT, [&] { return launch_rfft<T, T>(dm, plans, gin, wh, d, st); });
        const SpecOpParams sp = specop(cfg.incompressible != 0);
        run(KC_SPEC, [&] { return launch_spec_gradient<T>(dm, sp, vth, wh, wh, st); });
        // spec_precond gives -(alpha L)^-1 [P]: the inverse transform flips the sign
        run(KC_SPEC, [&] { return launch_spec_precond<T>(dm, sp, wh, wh, nullptr, st); });
        T* o[3] = {comp(out, 0), comp(out, 1), d == 3 ? comp(out, 2) : nullptr};
        run(KC_IRFFT, [&] { return launch_irfft<T>(dm, plans, wh, o, nullptr, -1.0 / Nt, d, st); });
    }

    // z = H0^-1 r approximately: GMRES from 0 on (alpha L)^-1 H0 z = (alpha L)^-1 r
    // (Arnoldi with modified Gram-Schmidt, Givens rotations on the host)
    void h0_precond(const T* q, T* z) {
        ensure_h0();
        const int m = kPcMaxit;
        T* bvec = pcv[0];
        precond_keep(q, bvec, false);  // (alpha L)^-1 [P] r, r = -q
        HIPCHK(hipMemsetAsync(z, 0, sizeof(T) * d * N, st));
        const double bn = std::sqrt(inner(bvec, bvec));
        if (bn == 0.0) return;
        std::vector<double> s1(1, 1.0 / bn - 1.0);
        run(KC_VEC, [&] { return launch_axpy<T>(bvec, s1.data(), bvec, pcv[0], vseg(), st); });
        std::vector<double> H((m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), e(m + 1, 0.0);
        auto Hij = [&](int i, int j) -> double& { return H[i * m + j]; };
        e[0] = bn;
        int its = 0;
        for (int j = 0; j < m; ++j) {
            h0_left(pcv[j], pcw);
            for (int i = 0; i <= j; ++i) {
                const double hij = inner(pcw, pcv[i]);
                Hij(i, j) = hij;
                const std::vector<double> mh(1, -hij);
                run(KC_VEC, [&] { return launch_axpy<T>(pcw, mh.data(), pcv[i], pcw, vseg(), st); });
            }
            const double hn = std::sqrt(inner(pcw, pcw));
            Hij(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
                Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
                Hij(i, j) = t;
            }
            const double den = std::hypot(Hij(j, j), Hij(j + 1, j));
            cs[j] = Hij(j, j) / den;
            sn[j] = Hij(j + 1, j) / den;
            Hij(j, j) = den;
            Hij(j + 1, j) = 0.0;
            e[j + 1] = -sn[j] * e[j];
            e[j] = cs[j] * e[j];
            its = j + 1;
            if (std::fabs(e[j + 1]) <= kPcTol * bn || hn == 0.0) break;
            const std::vector<double> sc(1, 1.0 / hn - 1.0);
            run(KC_VEC, [&] { return launch_axpy<T>(pcw, sc.data(), pcw, pcv[j + 1], vseg(), st); });
        }
        std::vector<double> y(its, 0.0);
        for (int i = its - 1; i >= 0; --i) {
            double t = e[i];
            for (int k2 = i + 1; k2 < its; ++k2) t -= Hij(i, k2) * y[k2];
            y[i] = t / Hij(i, i);
        }
        for (int i = 0; i < its; ++i) {
            const std::vector<double> yi(1, y[i]);
            run(KC_VEC, [&] { return launch_axpy<T>(z, yi.data(), pcv[i], z, vseg(), st); });
        }
    }

    // -- two-level -------------------------------------------------------------
    std::unique_ptr<Problem<T>> coarse;
    T *cv = nullptr, *cb = nullptr, *cy = nullptr, *cr = nullptr, *cp = nullptr, *cap = nullptr,
      *ct = nullptr, *cd = nullptr;
    const void* coarse_of = nullptr;  // fine velocity whose coarse state is current

    // coarse (d_out components) = restriction of fine (count fields of N)
    void restrict_to(const T* const* fine, T* const* out, int count, bool pow_half) {
        run(KC_RFFT, [&] { return launch_rfft<T, T>(dm, plans, fine, wh, count, st); });
        Problem<T>& C = *coarse;
        run(KC_SPEC, [&] {
            return launch_spec_resample<T>(dm, C.dm, wh, C.wh, count, 1, double(C.N) / double(N), st);
        });
        if (pow_half)
            run(KC_SPEC, [&] {
                return launch_spec_pow<T>(C.dm, C.specop(cfg.incompressible != 0), C.wh, C.wh, -0.5,
                                          1.0, 1, st);
            });
        run(KC_IRFFT, [&] { return launch_irfft<T>(C.dm, C.plans, C.wh, out, nullptr, 1.0 / C.N, count, st); });
    }

    void ensure_coarse() {
        if (coarse) return;
        for (int a = 0; a < d; ++a)
            if (cfg.n[a] % 2 != 0 || cfg.n[a] < 8)
                throw Error(GANMRES_EINVAL,
                            "the two-level preconditioner halves every axis: sizes must be even "
                            "and at least 8");
        ganmres_config cc = cfg;
        for (int a = 0; a < d; ++a) cc.n[a] = cfg.n[a] / 2;
        cc.checkpoint_every = 1;
        // the images passed here only fill the buffers; they are replaced below
        coarse.reset(new Problem<T>(cc, m0, m1, st));
        Problem<T>& C = *coarse;
        T* o0[1] = {C.m0};
        const T* i0[1] = {m0};
        restrict_to(i0, o0, 1, false);
        T* o1[1] = {C.m1};
        const T* i1[1] = {m1};
        restrict_to(i1, o1, 1, false);
        HIPCHK(hipMemcpyAsync(C.mstate(0), C.m0, sizeof(T) * C.N, hipMemcpyDeviceToDevice, st));
        cv = C.alloc_T(d * C.N);
        cb = C.alloc_T(d * C.N);
        cy = C.alloc_T(d * C.N);
        cr = C.alloc_T(d * C.N);
        cp = C.alloc_T(d * C.N);
        cap = C.alloc_T(d * C.N);
        ct = C.alloc_T(d * C.N);
        cd = C.alloc_T(d * C.N);
        coarse_of = nullptr;
    }

    // the coarse problem at the restriction of v (its state history)
    void coarse_at(const void* v) {
        ensure_coarse();
        Problem<T>& C = *coarse;
        const T* vin[3] = {comp(v, 0), comp(v, 1), d == 3 ? comp(v, 2) : nullptr};
        T* vo[3] = {C.comp(cv, 0), C.comp(cv, 1), d == 3 ? C.comp(cv, 2) : nullptr};
        restrict_to(vin, vo, d, false);
        C.prepare(cv, true);
        C.forward();
        C.fwd_valid = true;
        C.fwd_v = cv;
        coarse_of = v;
    }

    // out = (alpha L)^-1/2 [P] x on the coarse space (the modes outside it removed)
    static void reg_half(Problem<T>& C, const T* x, T* out) {
        const T* xin[3] = {C.comp(x, 0), C.comp(x, 1), C.d == 3 ? C.comp(x, 2) : nullptr};
        C.run(KC_RFFT, [&] { return launch_rfft<T, T>(C.dm, C.plans, xin, C.wh, C.d, C.st); });
        C.run(KC_SPEC, [&] {
            return launch_spec_pow<T>(C.dm, C.specop(C.cfg.incompressible != 0), C.wh, C.wh, -0.5,
                                      1.0, 1, C.st);
        });
        T* o[3] = {C.comp(out, 0), C.comp(out, 1), C.d == 3 ? C.comp(out, 2) : nullptr};
        C.run(KC_IRFFT, [&] { return launch_irfft<T>(C.dm, C.plans, C.wh, o, nullptr, 1.0 / C.N, C.d, C.st); });
    }

    // out = y + Hreg^-1/2 H_data,c Hreg^-1/2 y
    void coarse_op(const T* y, T* out) {
        Problem<T>& C = *coarse;
        reg_half(C, y, ct);
        C.gn_matvec(cv, ct, cd, true);
        reg_half(C, cd, out);
        const std::vector<double> one(1, 1.0);
        C.run(KC_VEC, [&] { return launch_axpy<T>(out, one.data(), y, out, C.vseg(), C.st); });
    }

    // z = M^-1 r for the two-level preconditioner at the velocity of the last coarse_at
    void twolevel_precond(const T* q, T* z) {
        Problem<T>& C = *coarse;
        precond_keep(q, z, false);  // (alpha L)^-1 [P] r
        // coarse right-hand side from q: b_q = Hreg^-1/2 restrict(q)
        const T* qin[3] = {comp(q, 0), comp(q, 1), d == 3 ? comp(q, 2) : nullptr};
        T* bo[3] = {C.comp(cb, 0), C.comp(cb, 1), d == 3 ? C.comp(cb, 2) : nullptr};
        restrict_to(qin, bo, d, true);
        // CG (no preconditioner) on the coarse operator
        HIPCHK(hipMemsetAsync(cy, 0, sizeof(T) * d * C.N, st));
        const double bn = std::sqrt(C.inner(cb, cb));
        if (bn > 0.0) {
            HIPCHK(hipMemcpyAsync(cr, cb, sizeof(T) * d * C.N, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(cp, cb, sizeof(T) * d * C.N, hipMemcpyDeviceToDevice, st));
            double rr = C.inner(cr, cr);
            for (int it = 0; it < kPcMaxit; ++it) {
                coarse_op(cp, cap);
                const double pap = C.inner(cp, cap);
                if (!(pap > 0.0)) break;
                const std::vector<double> a(1, rr / pap), ma(1, -rr / pap);
                C.run(KC_VEC, [&] { return launch_axpy<T>(cy, a.data(), cp, cy, C.vseg(), st); });
                C.run(KC_VEC, [&] { return launch_axpy<T>(cr, ma.data(), cap, cr, C.vseg(), st); });
                const double rr_new = C.inner(cr, cr);
                if (std::sqrt(rr_new) <= kPcTol * bn) break;
                const std::vector<double> be(1, rr_new / rr);
                C.run(KC_VEC, [&] { return launch_axpy<T>(cr, be.data(), cp, cp, C.vseg(), st); });
                rr = rr_new;
            }
        }
        // z -= prolong(Hreg^-1/2 (y_q - b_q))  (the low band replaces that of (alpha L)^-1 r)
        const std::vector<double> m1v(1, -1.0);
        C.run(KC_VEC, [&] { return launch_axpy<T>(cy, m1v.data(), cb, ct, C.vseg(), st); });
        const T* tin[3] = {C.comp(ct, 0), C.comp(ct, 1), d == 3 ? C.comp(ct, 2) : nullptr};
        run(KC_RFFT, [&] { return launch_rfft<T, T>(C.dm, C.plans, tin, C.wh, d, st); });
        run(KC_SPEC, [&] {
            return launch_spec_pow<T>(C.dm, C.specop(cfg.incompressible != 0), C.wh, C.wh, -0.5, 1.0,
                                      1, st);
        });
        run(KC_SPEC, [&] {
            return launch_spec_resample<T>(dm, C.dm, C.wh, wh, d, 0, double(N) / double(C.N), st);
        });
        T* zo[3] = {comp(z, 0), comp(z, 1), d == 3 ? comp(z, 2) : nullptr};
        const T* za[3] = {comp(z, 0), comp(z, 1), d == 3 ? comp(z, 2) : nullptr};
        run(KC_IRFFT, [&] { return launch_irfft<T>(dm, plans, wh, zo, za, -1.0 / N, d, st); });
    }

    // z = M^-1 r (r = -q) for preconditioner `which`, with the state of v current
    void apply_newton_pc(int which, const void* v, const T* q, T* z) {
        if (which == GANMRES_PC_H0RPC) {
            h0_precond(q, z);
        } else if (which == GANMRES_PC_2LRPCSYM) {
            if (coarse_of != v) coarse_at(v);
            twolevel_precond(q, z);
        } else {
            precond_keep(q, z, false);
        }
    }

    void newton_precond(int which, const void* v, const void* r, void* z) override {
        pre_g = nullptr;
        pre_spec_g = nullptr;
        check_newton_setup();
        if (which != GANMRES_PC_IREG && which != GANMRES_PC_H0RPC && which != GANMRES_PC_2LRPCSYM)
            throw Error(GANMRES_EINVAL, "unknown preconditioner");
        ensure_matvec_buffers();
        if (!qold) qold = pc_alloc(d * N);
        // q = -r
        const std::vector<double> m1v(1, -2.0);
        run(KC_VEC, [&] {
            return launch_axpy<T>(static_cast<const T*>(r), m1v.data(), static_cast<const T*>(r), qold,
                                  vseg(), st);
        });
        coarse_of = nullptr;  // the caller's v may have changed
        apply_newton_pc(which, v, qold, static_cast<T*>(z));
        HIPCHK(hipStreamSynchronize(st));
    }

    // <a, b>_h (FP64; single problem)
    double inner(const T* a, const T* bb) {
        run(KC_REDUCE, [&] { return launch_dot<T>(a, bb, vseg(), partial, dres + R_DOT, st); });
        return cell * fetch(R_DOT, 1)[0];
    }

    // One iteration of the inexact Gauss-Newton-Krylov method: PCG on
    // H_gn s = -g with the regulariser preconditioner ("ireg") to the forcing
    // tolerance min(1/2, sqrt(||g|| / ||g_0||)) (at most kCgMaxit
    // iterations), then Armijo backtracking from rho = 1.
    static constexpr int kCgMaxit = 50;
    double nk_g0norm = 0.0;
    void step_nk(const ganmres_solver_params& p, void* v, ganmres_step_info* info) {
        check_newton_setup();
        int ngrad = 0;
        T* V = rv(0);
        T* G = rg(0);
        if (!started) {
            start(p, v, V, G, ngrad);
            nk_g0norm = std::sqrt(inner(G, G));
        }
        T* S = rv(1);  // CG iterate, then the step
        T* Q = rg(1);  // -r
        T* Z = static_cast<T*>(gqb->p);
        T* Pd = static_cast<T*>(aa_r[0]->p);
        T* HP = static_cast<T*>(aa_q[0]->p);
        const double gn = std::sqrt(inner(G, G));
        const double tol = std::min(0.5, std::sqrt(gn / nk_g0norm));
        // CG from x = 0 on H x = b = -g.  Q holds -r (Q = g at the start) and
        // Z = M^-1 r, so <r, z> = -<Q, Z>.  With "ireg" (Z = -(alpha L)^-1 Q) the
        // usual update; with the inner-solve preconditioners the flexible one,
        // beta = <r_new - r_old, z_new> / <r_old, z_old>.  The state history of
        // V stays current through the iteration.
        const int pc = p.nk_precond;
        const bool flexible = pc != GANMRES_PC_IREG;
        if (flexible && !qold) qold = pc_alloc(d * N);
        if (pc == GANMRES_PC_2LRPCSYM) coarse_at(V);
        HIPCHK(hipMemsetAsync(S, 0, sizeof(T) * d * N, st));
        HIPCHK(hipMemcpyAsync(Q, G, sizeof(T) * d * N, hipMemcpyDeviceToDevice, st));
        apply_newton_pc(pc, V, Q, Z);
        HIPCHK(hipMemcpyAsync(Pd, Z, sizeof(T) * d * N, hipMemcpyDeviceToDevice, st));
        double rz = flexible ? -inner(Q, Z) : -gs_s[0];
        int its = 0;
        for (int it = 1; it <= kCgMaxit; ++it) {
            gn_matvec(V, Pd, HP);
            const double pHp = inner(Pd, HP);
            if (!(pHp > 0.0)) break;
            const double a = rz / pHp;
            const std::vector<double> av(1, a);
            run(KC_VEC, [&] { return launch_axpy<T>(S, av.data(), Pd, S, vseg(), st); });
            if (flexible)
                HIPCHK(hipMemcpyAsync(qold, Q, sizeof(T) * d * N, hipMemcpyDeviceToDevice, st));
            run(KC_VEC, [&] { return launch_axpy<T>(Q, av.data(), HP, Q, vseg(), st); });
            its = it;
            if (std::sqrt(inner(Q, Q)) <= tol * gn) break;
            apply_newton_pc(pc, V, Q, Z);
            const double rz_new = flexible ? -inner(Q, Z) : -gs_s[0];
            const double beta = flexible ? (rz_new + inner(qold, Z)) / rz : rz_new / rz;
            const std::vector<double> bv(1, beta);
            run(KC_VEC, [&] { return launch_axpy<T>(Z, bv.data(), Pd, Pd, vseg(), st); });
            rz = rz_new;
        }
        // line search from rho = 1 along s (regulariser as a quadratic in rho)
        if (vh_of != V) {
            spectrum_of(V);
            reg_s[0] = cell / double(Nt) * fetch(R_REG, 1)[0];
            reg_from_device = false;
        }
        if (umax_of != V) set_bounds(V, velocity_max(V));
        const double R0 = reg_s[0], um0 = umax;
        const double gs = inner(G, S);
        const T* sin_[3] = {comp(S, 0), comp(S, 1), d == 3 ? comp(S, 2) : nullptr};
        pre_spec_g = nullptr;
        run(KC_RFFT, [&] { return launch_rfft<T, T>(dm, plans, sin_, sk, d, st); });
        run(KC_REDUCE, [&] {
            return launch_spec_cross<T>(dm, specop(false), vh, sk, partial, dres + R_CROSS, st);
        });
        const double smx = velocity_max(S);
        const double* cr = fetch(R_CROSS, 2);
        const double cA = cell / double(Nt) * cr[0], cB = cell / double(Nt) * cr[1];
        T* q = static_cast<T*>(qb->p);
        double rho = 1.0, Jq = 0.0, Rq = R0;
        int trials = 0;
        bool ok = false;
        for (int t = 0; t <= p.max_backtracks; ++t) {
            ++trials;
            Rq = R0 + 2.0 * rho * cA + rho * rho * cB;
            const double bound = Jcur[0] + p.c_armijo * rho * gs;
            if (0.5 * alpha_s[0] * Rq >= bound) {
                rho *= 0.5;
                continue;
            }
            const std::vector<double> rv1(1, rho);
            run(KC_VEC, [&] { return launch_axpy<T>(V, rv1.data(), S, q, vseg(), st); });
            objective_trial(q, std::vector<double>(1, Rq), um0 + rho * smx);
            Jq = J_s[0];
            if (Jq < bound) {
                ok = true;
                break;
            }
            rho *= 0.5;
        }
        info[0].n_trials = trials;
        if (!ok) throw Error(GANMRES_ELINESEARCH, "Armijo condition not met");
        const std::vector<double> rv1(1, rho);
        run(KC_SPEC, [&] { return launch_spec_axpy<T>(dm, d, vh, rv1.data(), sk, st); });
        vh_of = q;
        reg_s[0] = Rq;
        reg_from_device = false;
        std::swap(ring_v[0], qb);  // v^{k+1} = q, forward solve kept
        gradient_async(rv(0), rg(0), true);  // J(q) is the accepted trial's
        J_pending = false;
        ++ngrad;
        info[0].step_kind = GANMRES_STEP_NEWTON;
        info[0].n_beta = its;
        finish_step(p, v, rv(0), rg(0), J_s, std::vector<double>(1, Jq), std::vector<double>(1, rho),
                    ngrad, info);
    }

    int count() const override { return nb; }

    // Deformation map y = x + h D (D^0 = 0, D^{j+1} = (X - i) + I[D^j](X)) and
    // det grad y with its (min, mean, max, std) per problem; det: device image
    // (nullable).  Uses the state's departure points of v.
    std::vector<std::unique_ptr<DevBuf>> dfm_bufs;
    void deformation(const void* v, void* det, double* stats) override {
        pre_g = nullptr;
        pre_spec_g = nullptr;
        prepare(v, false);
        // dX now belongs to v: a kept forward history of another velocity is void
        fwd_valid = false;
        adj_valid = false;
        y_valid = false;
        if (dfm_bufs.empty()) {
            for (int i = 0; i < 2 + d * d; ++i) {
                dfm_bufs.emplace_back(new DevBuf);
                dfm_bufs.back()->alloc(sizeof(T) * (i < 2 ? d * N : N));
            }
        }
        T* Da = static_cast<T*>(dfm_bufs[0]->p);
        T* Db = static_cast<T*>(dfm_bufs[1]->p);
        // D^1 = X - i
        HIPCHK(hipMemcpyAsync(Da, dX, sizeof(T) * d * N, hipMemcpyDeviceToDevice, st));
        for (int j = 1; j < cfg.nt; ++j) {
            for (int a = 0; a < d; ++a)
                run(KC_SL, [&] {
                    return launch_sl_step_add<T>(dm, comp(Da, a), dX, comp(dX, a), dbound,
                                                 comp(Db, a), st, tabX, tw(tabX_ok));
                });
            std::swap(Da, Db);
        }
        // J[a d + b] = dD_a / dx_b
        std::vector<const T*> J(d * d);
        const double one = 1.0;
        for (int a = 0; a < d; ++a)
            for (int bb = 0; bb < d; ++bb) {
                T* out = static_cast<T*>(dfm_bufs[2 + a * d + bb]->p);
                const T* f = comp(Da, a);
                run(KC_DERIV, [&] {
                    return launch_deriv_axis<T>(dm, plans, comp_axis(d, bb), &f, nullptr, &one, 1,
                                                0, out, st);
                });
                J[a * d + bb] = out;
            }
        double hc[3];
        for (int a = 0; a < d; ++a) hc[a] = h[comp_axis(d, a)];
        run(KC_REDUCE, [&] {
            return launch_det_stats<T>(J.data(), hc, d, sseg(), static_cast<T*>(det), partial,
                                       dres + R_GRAM, st);
        });
        const double* r = fetch(R_GRAM, 4 * nb);
        bool finite = true;
        for (int i = 0; i < nb; ++i) {
            const double mn = -r[i], mx = r[nb + i];
            const double m1 = r[2 * nb + i] / double(Nt), m2 = r[3 * nb + i] / double(Nt);
            const double var = std::max(0.0, m2 - m1 * m1);
            stats[4 * i + 0] = mn;
            stats[4 * i + 1] = 1.0 + m1;
            stats[4 * i + 2] = mx;
            stats[4 * i + 3] = std::sqrt(var);
            finite = finite && std::isfinite(mn) && std::isfinite(mx) && std::isfinite(m1);
        }
        if (!finite) throw Error(GANMRES_ENONFINITE, "non-finite deformation gradient");
    }
    void values(double* J, double* mis) const override {
        for (int i = 0; i < nb; ++i) {
            if (J) J[i] = J_s[i];
            if (mis) mis[i] = mis_s[i];
        }
    }

    // -- GA-NGMRES ----------------------------------------------------------
    void reset() override {
        pre_g = nullptr;
        pre_spec_g = nullptr;
        started = false;
        hist.clear();
        k = 0;
        rho_bar.assign(nb, 1.0);
    }

    T* rv(int slot) { return static_cast<T*>(ring_v[slot]->p); }
    T* rg(int slot) { return static_cast<T*>(ring_g[slot]->p); }
    T* ar(int slot) { return static_cast<T*>(aa_r[slot]->p); }
    T* aq(int slot) { return static_cast<T*>(aa_q[slot]->p); }

    // NGMRES keeps w+1 pairs (v, g) plus one being formed; AA keeps the current
    // and next (v, g) and w+1 pairs (r, q).
    void ensure_solver(int w, int acc) {
        if (wcap == w && acc_cap == acc) return;
        if (started) throw Error(GANMRES_EINVAL, "window or accelerator changed during a solve; reset first");
        const bool aa = acc == GANMRES_ACCEL_AA;
        const bool newton = acc == GANMRES_ACCEL_NK;
        ring_v.clear();
        ring_g.clear();
        for (int i = 0; i < (aa || newton ? 2 : w + 2); ++i) {
            ring_v.emplace_back(new DevBuf);
            ring_v.back()->alloc(sizeof(T) * d * N);
            ring_g.emplace_back(new DevBuf);
            ring_g.back()->alloc(sizeof(T) * d * N);
        }
        aa_r.clear();
        aa_q.clear();
        for (int i = 0; i < (aa ? w + 1 : (newton ? 1 : 0)); ++i) {
            aa_r.emplace_back(new DevBuf);
            aa_r.back()->alloc(sizeof(T) * d * N);
            aa_q.emplace_back(new DevBuf);
            aa_q.back()->alloc(sizeof(T) * d * N);
        }
        qb.reset(new DevBuf);
        qb->alloc(sizeof(T) * d * N);
        gqb.reset(new DevBuf);
        gqb->alloc(sizeof(T) * d * N);
        sb.reset(new DevBuf);
        sb->alloc(sizeof(T) * d * N);
        wcap = w;
        acc_cap = acc;
    }

    static bool is_fp(int k, const ganmres_solver_params& p) {
        if (p.sigma == 0) return true;
        const int m = k % (p.sigma + p.tau);
        return p.variant == GANMRES_VARIANT_ALT ? (m < p.tau) : (m >= p.sigma);
    }

    // Armijo line search from the current iterate (Vc, Gc, Jcur), each stacked
    // problem with its own step; the accepted trials are left in qb with
    // their forward solve kept (eqs. e:rpgd, e:armijo).  Along the line the
    // regulariser is a quadratic in rho:
    // R(v + rho s) = R(v) + 2 rho <v,L s>_h + rho^2 <s,L s>_h, and the spectrum
    // of the accepted trial is v^ + rho s^; trials need no transform of their
    // own.  Returns the accepted steps; Jq receives J(q) per problem.
    std::vector<double> line_search(T* Vc, T* Gc, const ganmres_solver_params& p,
                                    ganmres_step_info* info, std::vector<double>& Jq) {
        T* q = static_cast<T*>(qb->p);
        T* s = static_cast<T*>(sb->p);
        if (vh_of != Vc) {
            spectrum_of(Vc);
            const double* r = fetch(R_REG, nb);
            for (int i = 0; i < nb; ++i) reg_s[i] = cell / double(Nt) * r[i];
            reg_from_device = false;
        }
        if (umax_of != Vc) set_bounds(Vc, velocity_max(Vc));
        const std::vector<double> R0 = reg_s;
        const double um0 = umax;
        if (pre_g != Gc) precond_keep(Gc, s, true);
        pre_g = nullptr;
        pre_spec_g = nullptr;
        std::vector<double> cA(nb), cB(nb);
        for (int i = 0; i < nb; ++i) {
            cA[i] = cell / double(Nt) * crossA[i];
            cB[i] = cell / double(Nt) * crossB[i];
        }
        std::vector<double> rho(rho_bar), Rq(R0);
        std::vector<int> trials(nb, 0);
        std::vector<char> done(nb, 0);
        Jq.assign(nb, 0.0);
        int open = nb;
        // the classes of a group handle backtrack together until all have
        // accepted (a class with nothing left to decide launches nothing)
        for (int t = 0; t <= p.max_backtracks && group_any(open > 0); ++t) {
            std::vector<double> bound(nb, 0.0);
            bool transport = false;
            for (int i = 0; i < nb; ++i) {
                if (done[i]) continue;
                Rq[i] = R0[i] + 2.0 * rho[i] * cA[i] + rho[i] * rho[i] * cB[i];
                bound[i] = Jcur[i] + p.c_armijo * rho[i] * gs_s[i];
                ++trials[i];
                // J(q) = mismatch + alpha/2 R(q) with mismatch >= 0: a trial
                // whose regulariser term alone reaches the Armijo bound fails
                // whatever its transport gives (the same expression as in
                // finish_J, so the decision is the one the full evaluation
                // would take)
                if (0.5 * alpha_s[i] * Rq[i] >= bound[i]) {
                    rho[i] *= 0.5;
                    bound[i] = -INFINITY;  // decided
                } else {
                    transport = true;
                }
            }
            if (!transport) continue;
            run(KC_VEC, [&] { return launch_axpy<T>(Vc, rho.data(), s, q, vseg(), st); });
            double rmax = 0.0;
            for (int i = 0; i < nb; ++i) rmax = std::max(rmax, rho[i]);
            objective_trial(q, Rq, um0 + rmax * smax);
            for (int i = 0; i < nb; ++i) {
                if (done[i] || bound[i] == -INFINITY) continue;
                if (J_s[i] < bound[i]) {
                    Jq[i] = J_s[i];
                    rho_bar[i] = (trials[i] == 1) ? 2.0 * rho[i] : rho[i];
                    if (p.rho_cap > 0.0) rho_bar[i] = std::min(rho_bar[i], p.rho_cap);
                    done[i] = 1;
                    --open;
                } else {
                    rho[i] *= 0.5;
                }
            }
        }
        for (int i = 0; i < nb; ++i) info[i].n_trials = trials[i];
        if (open > 0) throw Error(GANMRES_ELINESEARCH, "Armijo condition not met");
        run(KC_SPEC, [&] { return launch_spec_axpy<T>(dm, d, vh, rho.data(), sk, st); });
        vh_of = q;
        reg_s = Rq;
        reg_from_device = false;
        return rho;
    }

    // least-squares coefficients per problem from the FP64 Gram matrices of
    // vecs[0..K) (one reduction over the K vectors and one fetch):
    // beta[i * (K-1) ..] is the solution of problem i; lsq_fb[i] records
    // whether its solve fell back to the pseudo-inverse
    std::vector<char> lsq_fb;
    std::vector<double> gram_lsq(const std::vector<const T*>& vecs) {
        const int K = (int)vecs.size();
        const int np = K * (K + 1) / 2;
        std::vector<double> G(np * nb);
        run(KC_REDUCE, [&] {
            return launch_gram<T>(vecs.data(), K, vseg(), partial, dres + R_GRAM, st);
        });
        const double* r = fetch(R_GRAM, np * nb);
        for (int x = 0; x < np * nb; ++x) G[x] = r[x];
        std::vector<double> beta;
        std::vector<double> Gi(K * K);
        lsq_fb.assign(nb, 0);
        for (int i = 0; i < nb; ++i) {
            int qi = 0;
            for (int a = 0; a < K; ++a)
                for (int bb = a; bb < K; ++bb, ++qi) Gi[a * K + bb] = Gi[bb * K + a] = G[qi * nb + i];
            bool fb = false;
            const std::vector<double> bi = lsq_from_gram(K, Gi, &fb);
            lsq_fb[i] = fb ? 1 : 0;
            for (double x : bi)
                if (!std::isfinite(x)) throw Error(GANMRES_ELSQ, "non-finite least-squares coefficients");
            beta.insert(beta.end(), bi.begin(), bi.end());
        }
        return beta;
    }

    // out = q + sum_k coef_i[k] (q - xs[k]) with the coefficients of problem i
    // at beta[i * K + k]
    void combine(const T* q, const std::vector<const T*>& xs, const std::vector<double>& beta,
                 int K, T* out) {
        for (int kk = 0; kk < K; ++kk)
            for (int i = 0; i < nb; ++i) hup[kk * nb + i] = beta[i * K + kk];
        HIPCHK(hipMemcpyAsync(coef_dev, hup, sizeof(double) * K * nb, hipMemcpyHostToDevice, st));
        run(KC_VEC, [&] { return launch_combine<T>(q, xs.data(), coef_dev, K, out, vseg(), st); });
        // hup is next written by the following step's mixing, after several
        // synchronisations of the stream: the copy has run by then
    }

    void finish_step(const ganmres_solver_params& p, void* v, T* Vn, T* Gn,
                     const std::vector<double>& Jnew, const std::vector<double>& Jq,
                     const std::vector<double>& rho, int ngrad, ganmres_step_info* info) {
        ++k;
        run(KC_REDUCE, [&] { return launch_maxabs<T>(Gn, vseg(), partial, dres + R_MAX, st); });
        HIPCHK(hipMemcpyAsync(v, Vn, sizeof(T) * d * N, hipMemcpyDeviceToDevice, st));
        // the next iteration starts with the direction of g^{k+1}: launched
        // now, it reaches the host with this synchronisation
        const bool prefetch = k < p.n_iter;
        if (prefetch) precond_launch(Gn, sb->p, true);
        stream_sync(st);
        if (prefetch) {
            precond_collect(true);
            pre_g = Gn;
        }
        if (J_pending) resolve_J();  // the stream has passed the mismatch
        const std::vector<double>& Jv = Jnew.empty() ? J_s : Jnew;
        const std::vector<double> ginf(hres + R_MAX, hres + R_MAX + nb);
        bool finite = true;
        for (int i = 0; i < nb; ++i) {
            Jcur[i] = Jv[i];
            info[i].k = k;
            info[i].J = Jv[i];
            info[i].J_q = Jq[i];
            info[i].ginf = ginf[i];
            info[i].g0inf = g0inf[i];
            info[i].rho = rho[i];
            info[i].n_grad = ngrad;
            info[i].stop = (ginf[i] <= p.eps_rel * g0inf[i]) || (k >= p.n_iter);
            finite = finite && std::isfinite(Jv[i]) && std::isfinite(ginf[i]);
        }
        if (!finite) throw Error(GANMRES_ENONFINITE, "non-finite objective or gradient");
    }

    void start(const ganmres_solver_params& p, void* v, T* V0, T* G0, int& ngrad) {
        HIPCHK(hipMemcpyAsync(V0, v, sizeof(T) * d * N, hipMemcpyDeviceToDevice, st));
        gradient(V0, G0, false);
        ++ngrad;
        Jcur = J_s;
        g0inf = maxabs(G0);
        for (int i = 0; i < nb; ++i)
            if (!std::isfinite(Jcur[i]) || !std::isfinite(g0inf[i]))
                throw Error(GANMRES_ENONFINITE, "non-finite objective or gradient at v^0");
        k = 0;
        rho_bar.assign(nb, 1.0);
        started = true;
    }

    void step(const ganmres_solver_params& p, void* v, ganmres_step_info* info) override {
        ensure_solver(p.accel == GANMRES_ACCEL_NK ? 0 : p.w, p.accel);
        for (int i = 0; i < nb; ++i) info[i] = ganmres_step_info{};
        if (p.accel == GANMRES_ACCEL_AA) step_aa(p, v, info);
        else if (p.accel == GANMRES_ACCEL_NK) step_nk(p, v, info);
        else step_ngmres(p, v, info);
    }

    // One iteration of GA-NGMRES(w; sigma, tau) (Alg. 3).
    void step_ngmres(const ganmres_solver_params& p, void* v, ganmres_step_info* info) {
        int ngrad = 0;
        if (!started) {
            start(p, v, rv(0), rg(0), ngrad);
            hist.assign(1, 0);
        }
        const int cur = hist.back();
        std::vector<double> Jq;
        const std::vector<double> rho = line_search(rv(cur), rg(cur), p, info, Jq);
        T* q = static_cast<T*>(qb->p);
        T* gq = static_cast<T*>(gqb->p);
        // J(q) is the accepted trial's: no need to wait for it; in an FP step
        // g(q) is the next iterate's gradient, whose direction comes next
        gradient_async(q, gq, true, false, is_fp(k, p));
        J_pending = false;
        ++ngrad;
        // the free slot (not in the window)
        int slot = -1;
        for (int i = 0; i < (int)ring_v.size(); ++i)
            if (std::find(hist.begin(), hist.end(), i) == hist.end()) {
                slot = i;
                break;
            }
        std::vector<double> Jnew;
        if (is_fp(k, p)) {
            std::swap(ring_v[slot], qb);
            std::swap(ring_g[slot], gqb);
            Jnew = Jq;
            for (int i = 0; i < nb; ++i) info[i].step_kind = GANMRES_STEP_FP;
        } else {
            const int wk = std::min(k, p.w);
            std::vector<const T*> vecs(wk + 2);
            vecs[0] = gq;
            for (int i = 0; i <= wk; ++i) vecs[i + 1] = rg(hist[hist.size() - 1 - i]);
            const std::vector<double> beta = gram_lsq(vecs);
            std::vector<const T*> xs(wk + 1);
            for (int i = 0; i <= wk; ++i) xs[i] = rv(hist[hist.size() - 1 - i]);
            combine(q, xs, beta, wk + 1, rv(slot));
            gradient_async(rv(slot), rg(slot), false, false, true);  // J taken up in finish_step
            ++ngrad;
            for (int i = 0; i < nb; ++i) {
                info[i].step_kind = GANMRES_STEP_NGMRES;
                info[i].n_beta = wk + 1;
                info[i].lsq_fallback = lsq_fb[i];
                for (int j = 0; j <= wk && j <= GANMRES_MAX_WINDOW; ++j)
                    info[i].beta[j] = beta[i * (wk + 1) + j];
            }
        }
        hist.push_back(slot);
        while ((int)hist.size() > p.w + 1) hist.pop_front();
        finish_step(p, v, rv(slot), rg(slot), Jnew, Jq, rho, ngrad, info);
    }

    // One iteration of GA-AA(w; sigma, tau): Alg. 2 with the alternation of
    // Alg. 3.  Ring slots hold (r, q) = (v - q(v), q(v)); slots 0/1 of the
    // (v, g) ring alternate as the current and the next iterate.
    void step_aa(const ganmres_solver_params& p, void* v, ganmres_step_info* info) {
        int ngrad = 0;
        if (!started) {
            start(p, v, rv(0), rg(0), ngrad);
            aa_cur = 0;
            hist.clear();
        }
        T* Vc = rv(aa_cur);
        T* Gc = rg(aa_cur);
        const int nxt = 1 - aa_cur;
        std::vector<double> Jq;
        const std::vector<double> rho = line_search(Vc, Gc, p, info, Jq);
        T* q = static_cast<T*>(qb->p);
        const int wk = std::min(k, p.w);
        // the free (r, q) slot
        int slot = -1;
        for (int i = 0; i < (int)aa_r.size(); ++i)
            if (std::find(hist.begin(), hist.end(), i) == hist.end()) {
                slot = i;
                break;
            }
        if (slot >= 0) {
            const std::vector<double> minus(nb, -1.0);
            run(KC_VEC, [&] { return launch_axpy<T>(Vc, minus.data(), q, ar(slot), vseg(), st); });
            HIPCHK(hipMemcpyAsync(aq(slot), q, sizeof(T) * d * N, hipMemcpyDeviceToDevice, st));
        }
        std::vector<double> Jnew;
        if (is_fp(k, p) || wk == 0) {
            // v^{k+1} = q: the trial buffer becomes the next iterate, and its
            // forward solve from the line search is reused
            std::swap(ring_v[nxt], qb);
            gradient_async(rv(nxt), rg(nxt), true, false, true);
            J_pending = false;
            Jnew = J_s;
            for (int i = 0; i < nb; ++i) info[i].step_kind = GANMRES_STEP_FP;
        } else {
            std::vector<const T*> vecs(wk + 1);
            vecs[0] = ar(slot);
            for (int i = 1; i <= wk; ++i) vecs[i] = ar(hist[hist.size() - i]);
            const std::vector<double> xi = gram_lsq(vecs);
            std::vector<const T*> xs(wk);
            for (int i = 1; i <= wk; ++i) xs[i - 1] = aq(hist[hist.size() - i]);
            combine(q, xs, xi, wk, rv(nxt));
            gradient_async(rv(nxt), rg(nxt), false, false, true);  // J taken up in finish_step
            for (int i = 0; i < nb; ++i) {
                info[i].step_kind = GANMRES_STEP_AA;
                info[i].n_beta = wk;
                info[i].lsq_fallback = lsq_fb[i];
                for (int j = 0; j < wk && j <= GANMRES_MAX_WINDOW; ++j) info[i].beta[j] = xi[i * wk + j];
            }
        }
        ++ngrad;
        if (slot >= 0) {
            hist.push_back(slot);
            while ((int)hist.size() > p.w) hist.pop_front();
        }
        aa_cur = nxt;
        finish_step(p, v, rv(nxt), rg(nxt), Jnew, Jq, rho, ngrad, info);
    }
};

// A group handle: batches of 2-D problems of different grid sizes ("size
// classes", each a stacked batch handle of its own) that run every phase
// together: the classes execute as cooperative tasks (coop_run) and their
// launches of one kernel family are issued as one launch.  Velocities,
// images and per-problem results are the classes' back to back.
template <typename T>
class GroupProblem : public ProblemBase {
   public:
    std::vector<std::unique_ptr<Problem<T>>> cls;
    std::vector<size_t> voff, ioff;  // bytes of the velocities / images before class c
    std::vector<int> poff;           // problems before class c
    int total = 0;
    hipStream_t st;
    CoopStats stats;

    GroupProblem(const ganmres_config& cfg, int nclass, const int* shapes, const int* counts,
                 const double* alpha, const void* const* m0, const void* const* m1, hipStream_t s)
        : st(s) {
        size_t vo = 0, io = 0;
        for (int c = 0; c < nclass; ++c) {
            ganmres_config cc = cfg;
            cc.n[0] = shapes[2 * c];
            cc.n[1] = shapes[2 * c + 1];
            cc.n[2] = 1;
            cls.emplace_back(new Problem<T>(cc, m0[c], m1[c], s, counts[c], alpha ? alpha + total : nullptr));
            voff.push_back(vo);
            ioff.push_back(io);
            poff.push_back(total);
            const size_t pts = (size_t)counts[c] * cc.n[0] * cc.n[1];
            vo += 2 * pts * sizeof(T);
            io += pts * sizeof(T);
            total += counts[c];
        }
    }
    const void* vp(const void* v, int c) const { return static_cast<const char*>(v) + voff[c]; }
    void* vp(void* v, int c) const { return static_cast<char*>(v) + voff[c]; }

    // f(c) for every class, the classes' launches merged
    template <typename F>
    void each(F&& f) {
        std::vector<std::function<void()>> fns;
        for (int c = 0; c < (int)cls.size(); ++c) fns.push_back([&f, c] { f(c); });
        coop_run(fns, st, &stats);
    }

    double objective(const void* v, bool keep, double* mismatch) override {
        std::vector<double> J(cls.size()), M(cls.size());
        each([&](int c) { J[c] = cls[c]->objective(vp(v, c), keep, &M[c]); });
        double jt = 0.0, mt = 0.0;
        for (size_t c = 0; c < cls.size(); ++c) {
            jt += J[c];
            mt += M[c];
        }
        if (mismatch) *mismatch = mt;
        return jt;
    }
    double gradient(const void* v, void* g, bool reuse) override {
        std::vector<double> J(cls.size());
        each([&](int c) { J[c] = cls[c]->gradient(vp(v, c), vp(g, c), reuse); });
        double jt = 0.0;
        for (double x : J) jt += x;
        return jt;
    }
    double precond(const void* g, void* s) override {
        std::vector<double> G(cls.size());
        each([&](int c) { G[c] = cls[c]->precond(vp(g, c), vp(s, c)); });
        double t = 0.0;
        for (double x : G) t += x;
        return t;
    }
    void step(const ganmres_solver_params& p, void* v, ganmres_step_info* info) override {
        if (p.accel == GANMRES_ACCEL_NK)
            throw Error(GANMRES_EINVAL, "the Newton-Krylov baseline runs on single problems");
        each([&](int c) { cls[c]->step(p, vp(v, c), info + poff[c]); });
    }
    int count() const override { return total; }
    void deformation(const void* v, void* det, double* st4) override {
        each([&](int c) {
            cls[c]->deformation(vp(v, c), det ? static_cast<char*>(det) + ioff[c] : nullptr,
                                st4 + 4 * poff[c]);
        });
    }
    void hessian_matvec(const void*, const void*, void*) override {
        throw Error(GANMRES_EINVAL, "the Gauss-Newton Hessian needs a single problem");
    }
    void newton_precond(int, const void*, const void*, void*) override {
        throw Error(GANMRES_EINVAL, "the Newton-step preconditioners need a single problem");
    }
    void values(double* J, double* mis) const override {
        for (size_t c = 0; c < cls.size(); ++c)
            cls[c]->values(J ? J + poff[c] : nullptr, mis ? mis + poff[c] : nullptr);
    }
    void reset() override {
        for (auto& p : cls) p->reset();
    }
    void get_field(int which, int j, void* out) override {
        each([&](int c) { cls[c]->get_field(which, j, static_cast<char*>(out) + ioff[c]); });
    }
    long long workspace_bytes() const override {
        long long b = 0;
        for (auto& p : cls) b += p->workspace_bytes();
        return b;
    }
    void timing_flush() override {}
};

}  // namespace gan

struct ganmres_handle {
    std::unique_ptr<gan::ProblemBase> impl;
    std::string err;
    int dtype;
};

static thread_local std::string g_create_error;
std::string& gan::handle_free_error() { return g_create_error; }

template <typename F>
static int guarded(ganmres_handle* h, F&& f) {
    try {
        f();
        if (h) h->err.clear();
        return GANMRES_OK;
    } catch (const gan::Error& e) {
        if (h) h->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (h) h->err = "host allocation failed";
        return GANMRES_ENOMEM;
    } catch (...) {
        if (h) h->err = "unexpected error";
        return GANMRES_EDEVICE;
    }
}

// the Python binding mirrors these layouts
static_assert(sizeof(ganmres_config) == 48, "ganmres_config layout");
static_assert(sizeof(ganmres_solver_params) == 72, "ganmres_solver_params layout");
static_assert(sizeof(ganmres_step_info) == 592, "ganmres_step_info layout");

static int create_impl(const ganmres_config* cfg, int count, const double* alpha, const void* m0,
                       const void* m1, void* stream, ganmres_handle** out) {
    if (!cfg || !m0 || !m1 || !out) {
        g_create_error = "null argument";
        return GANMRES_EINVAL;
    }
    *out = nullptr;
    const ganmres_config& c = *cfg;
    std::string why;
    if (count < 1 || count > gan::kMaxSeg) why = "count must be in [1, 64]";
    if (why.empty() && count > 1 && c.dim != 2) why = "batches stack 2-D problems";
    for (int i = 0; alpha && i < count && why.empty(); ++i)
        if (!(alpha[i] > 0.0)) why = "alpha must be > 0";
    {
        const std::string cw = gan::config_error(c);
        if (!cw.empty()) why = cw;
    }
    if (!why.empty()) {
        g_create_error = why;
        return GANMRES_EINVAL;
    }
    auto* h = new ganmres_handle;
    h->dtype = c.dtype;
    const int rc = guarded(h, [&] {
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (c.dtype == GANMRES_F32) h->impl.reset(new gan::Problem<float>(c, m0, m1, st, count, alpha));
        else h->impl.reset(new gan::Problem<double>(c, m0, m1, st, count, alpha));
    });
    if (rc != GANMRES_OK) {
        g_create_error = h->err;
        delete h;
        return rc;
    }
    *out = h;
    return GANMRES_OK;
}

static int create_group_impl(const ganmres_config* cfg, int nclass, const int* shapes,
                             const int* counts, const double* alpha, const void* const* m0,
                             const void* const* m1, void* stream, ganmres_handle** out) {
    if (!cfg || !shapes || !counts || !m0 || !m1 || !out) {
        g_create_error = "null argument";
        return GANMRES_EINVAL;
    }
    *out = nullptr;
    std::string why;
    if (cfg->dim != 2) why = "a group holds 2-D problems";
    if (why.empty() && (nclass < 1 || nclass > gan::kMaxClasses)) why = "nclass must be in [1, 16]";
    int total = 0;
    for (int c = 0; why.empty() && c < nclass; ++c) {
        if (counts[c] < 1 || counts[c] > gan::kMaxSeg) why = "every class count must be in [1, 64]";
        if (!m0[c] || !m1[c]) why = "null image";
        ganmres_config cc = *cfg;
        cc.n[0] = shapes[2 * c];
        cc.n[1] = shapes[2 * c + 1];
        cc.n[2] = 1;
        const std::string cw = gan::config_error(cc);
        if (why.empty() && !cw.empty()) why = cw;
        total += counts[c];
    }
    for (int i = 0; why.empty() && alpha && i < total; ++i)
        if (!(alpha[i] > 0.0)) why = "alpha must be > 0";
    if (!why.empty()) {
        g_create_error = why;
        return GANMRES_EINVAL;
    }
    auto* h = new ganmres_handle;
    h->dtype = cfg->dtype;
    const int rc = guarded(h, [&] {
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (cfg->dtype == GANMRES_F32)
            h->impl.reset(new gan::GroupProblem<float>(*cfg, nclass, shapes, counts, alpha, m0, m1, st));
        else
            h->impl.reset(new gan::GroupProblem<double>(*cfg, nclass, shapes, counts, alpha, m0, m1, st));
    });
    if (rc != GANMRES_OK) {
        g_create_error = h->err;
        delete h;
        return rc;
    }
    *out = h;
    return GANMRES_OK;
}

extern "C" {

int ganmres_create_group(const ganmres_config* cfg, int nclass, const int* shapes,
                         const int* counts, const double* alpha, const void* const* m0,
                         const void* const* m1, void* stream, ganmres_handle** out) {
    return create_group_impl(cfg, nclass, shapes, counts, alpha, m0, m1, stream, out);
}

int ganmres_tile_autotune(const ganmres_handle* h, int cls, int* points_per_thread, double* us) {
    if (!h || !points_per_thread) return GANMRES_EINVAL;
    auto report = [&](auto* p) {
        *points_per_thread = p->tile_choice;
        if (us)
            for (int i = 0; i < 3; ++i) us[i] = p->tile_us[i];
    };
    if (auto* g = dynamic_cast<const gan::GroupProblem<float>*>(h->impl.get())) {
        if (cls < 0 || cls >= (int)g->cls.size()) return GANMRES_EINVAL;
        report(g->cls[cls].get());
    } else if (auto* g = dynamic_cast<const gan::GroupProblem<double>*>(h->impl.get())) {
        if (cls < 0 || cls >= (int)g->cls.size()) return GANMRES_EINVAL;
        report(g->cls[cls].get());
    } else if (auto* p = dynamic_cast<const gan::Problem<float>*>(h->impl.get())) {
        if (cls != 0) return GANMRES_EINVAL;
        report(p);
    } else if (auto* p = dynamic_cast<const gan::Problem<double>*>(h->impl.get())) {
        if (cls != 0) return GANMRES_EINVAL;
        report(p);
    } else {
        return GANMRES_EINVAL;
    }
    return GANMRES_OK;
}

int ganmres_group_launches(const ganmres_handle* h, long long* submitted, long long* issued) {
    if (!h || !submitted || !issued) return GANMRES_EINVAL;
    const gan::CoopStats* s = nullptr;
    if (auto* g = dynamic_cast<const gan::GroupProblem<float>*>(h->impl.get())) s = &g->stats;
    if (auto* g = dynamic_cast<const gan::GroupProblem<double>*>(h->impl.get())) s = &g->stats;
    if (!s) return GANMRES_EINVAL;
    *submitted = s->submitted;
    *issued = s->issued;
    return GANMRES_OK;
}

int ganmres_create(const ganmres_config* cfg, const void* m0, const void* m1, void* stream,
                   ganmres_handle** out) {
    return create_impl(cfg, 1, nullptr, m0, m1, stream, out);
}

int ganmres_create_batch(const ganmres_config* cfg, int count, const double* alpha, const void* m0,
                         const void* m1, void* stream, ganmres_handle** out) {
    return create_impl(cfg, count, alpha, m0, m1, stream, out);
}

int ganmres_batch_count(const ganmres_handle* h) { return h ? h->impl->count() : 0; }

int ganmres_batch_values(ganmres_handle* h, double* J, double* mismatch) {
    if (!h || (!J && !mismatch)) return GANMRES_EINVAL;
    return guarded(h, [&] { h->impl->values(J, mismatch); });
}

int ganmres_lsq(int K, const double* G, double* beta, int* fallback) {
    if (K < 2 || K > gan::kMaxGram || !G || !beta) return GANMRES_EINVAL;
    try {
        std::vector<double> Gv(G, G + (size_t)K * K);
        for (int a = 0; a < K; ++a)
            for (int b = 0; b < K; ++b)
                if (!std::isfinite(Gv[a * K + b]) || Gv[a * K + b] != Gv[b * K + a]) return GANMRES_EINVAL;
        bool fb = false;
        const std::vector<double> x = gan::lsq_from_gram(K, Gv, &fb);
        for (int i = 0; i < K - 1; ++i) {
            if (!std::isfinite(x[i])) return GANMRES_ELSQ;
            beta[i] = x[i];
        }
        if (fallback) *fallback = fb ? 1 : 0;
        return GANMRES_OK;
    } catch (...) {
        return GANMRES_ENOMEM;
    }
}

int ganmres_destroy(ganmres_handle* h) {
    delete h;
    return GANMRES_OK;
}

const char* ganmres_last_error(const ganmres_handle* h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

int ganmres_eval_objective(ganmres_handle* h, const void* v, int keep_history, double* J,
                           double* mismatch) {
    if (!h || !v || !J) return GANMRES_EINVAL;
    int rc = guarded(h, [&] { *J = h->impl->objective(v, keep_history != 0, mismatch); });
    if (rc == GANMRES_OK && !std::isfinite(*J)) {
        h->err = "non-finite objective";
        rc = GANMRES_ENONFINITE;
    }
    return rc;
}

int ganmres_eval_gradient(ganmres_handle* h, const void* v, void* g, int reuse_forward, double* J) {
    if (!h || !v || !g || v == g) {
        if (h) h->err = "invalid arguments";
        return GANMRES_EINVAL;
    }
    double Jv = 0.0;
    int rc = guarded(h, [&] { Jv = h->impl->gradient(v, g, reuse_forward != 0); });
    if (J) *J = Jv;
    if (rc == GANMRES_OK && !std::isfinite(Jv)) {
        h->err = "non-finite objective";
        rc = GANMRES_ENONFINITE;
    }
    return rc;
}

int ganmres_apply_precond(ganmres_handle* h, const void* g, void* s, double* gs) {
    if (!h || !g || !s) return GANMRES_EINVAL;
    double x = 0.0;
    const int rc = guarded(h, [&] { x = h->impl->precond(g, s); });
    if (gs) *gs = x;
    return rc;
}

int ganmres_step(ganmres_handle* h, const ganmres_solver_params* p, void* v,
                 ganmres_step_info* info) {
    if (!h || !p || !v) return GANMRES_EINVAL;
    const bool mixing = p->accel != GANMRES_ACCEL_NK;  // w, sigma and tau are used
    if (!mixing && p->nk_precond != GANMRES_PC_IREG && p->nk_precond != GANMRES_PC_H0RPC &&
        p->nk_precond != GANMRES_PC_2LRPCSYM) {
        h->err = "unknown Newton-Krylov preconditioner";
        return GANMRES_EINVAL;
    }
    if ((mixing && (p->w < 0 || p->w > GANMRES_MAX_WINDOW || p->sigma < 0 || p->tau < 0 ||
                    (p->sigma + p->tau) == 0)) ||
        p->n_iter < 1 || p->max_backtracks < 0 ||
        (p->accel != GANMRES_ACCEL_NGMRES && p->accel != GANMRES_ACCEL_AA &&
         p->accel != GANMRES_ACCEL_NK)) {
        h->err = "invalid solver parameters";
        return GANMRES_EINVAL;
    }
    std::vector<ganmres_step_info> local;
    return guarded(h, [&] {
        if (!info) {
            local.resize(h->impl->count());
            h->impl->step(*p, v, local.data());
        } else {
            h->impl->step(*p, v, info);
        }
    });
}

int ganmres_deformation(ganmres_handle* h, const void* v, void* det, double* stats) {
    if (!h || !v || !stats) {
        if (h) h->err = "invalid arguments";
        return GANMRES_EINVAL;
    }
    return guarded(h, [&] { h->impl->deformation(v, det, stats); });
}

int ganmres_hessian_matvec(ganmres_handle* h, const void* v, const void* vt, void* out) {
    if (!h || !v || !vt || !out || vt == out || v == out) {
        if (h) h->err = "invalid arguments";
        return GANMRES_EINVAL;
    }
    return guarded(h, [&] { h->impl->hessian_matvec(v, vt, out); });
}

int ganmres_newton_precond(ganmres_handle* h, int which, const void* v, const void* r, void* z) {
    if (!h || !v || !r || !z || r == z || v == z) {
        if (h) h->err = "invalid arguments";
        return GANMRES_EINVAL;
    }
    return guarded(h, [&] { h->impl->newton_precond(which, v, r, z); });
}

int ganmres_solver_reset(ganmres_handle* h) {
    if (!h) return GANMRES_EINVAL;
    return guarded(h, [&] { h->impl->reset(); });
}

int ganmres_get_field(ganmres_handle* h, int which, int j, void* out) {
    if (!h || !out) return GANMRES_EINVAL;
    return guarded(h, [&] { h->impl->get_field(which, j, out); });
}

int ganmres_timing_enable(ganmres_handle* h, int on) {
    if (!h) return GANMRES_EINVAL;
    return guarded(h, [&] {
        if (!on) h->impl->timing_flush();
        h->impl->timing = on != 0;
    });
}

int ganmres_timing_select(ganmres_handle* h, unsigned mask) {
    if (!h) return GANMRES_EINVAL;
    return guarded(h, [&] {
        h->impl->timing_flush();
        h->impl->tmask = mask;
    });
}

int ganmres_timing_reset(ganmres_handle* h) {
    if (!h) return GANMRES_EINVAL;
    return guarded(h, [&] {
        h->impl->timing_flush();
        for (int i = 0; i < gan::KC_COUNT; ++i) {
            h->impl->tms[i] = 0.0;
            h->impl->tcount[i] = 0;
        }
    });
}

int ganmres_timing_get(ganmres_handle* h, int kernel, double* ms, long long* launches) {
    if (!h || kernel < 0 || kernel >= gan::KC_COUNT) return GANMRES_EINVAL;
    return guarded(h, [&] {
        h->impl->timing_flush();
        if (ms) *ms = h->impl->tms[kernel];
        if (launches) *launches = h->impl->tcount[kernel];
    });
}

int ganmres_kernel_count(void) { return gan::KC_COUNT; }

const char* ganmres_kernel_name(int kernel) {
    if (kernel < 0 || kernel >= gan::KC_COUNT) return "";
    return gan::kKernelNames[kernel];
}

long long ganmres_workspace_bytes(const ganmres_handle* h) {
    return h ? h->impl->workspace_bytes() : 0;
}

}  // extern "C"
