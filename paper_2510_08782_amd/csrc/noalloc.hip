// The objective J(v) without a handle and without any device allocation:
// every intermediate field lives in one file-scope device array, `scratch`,
// of kScratchBytes per GPU (held until the process ends).  The same kernels
// as ganmres_eval_objective run, on pointers carved out of that array.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/ganmres.h"
#include "config.hpp"
#include "fft_core.hpp"
#include "launch.hpp"

namespace gan {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, taken once per device with that
// device current.  In host code the array's name is not a device address.
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// exp(-2 pi i m / L) per axis, computed in FP64 on the device (sincospi),
// stored in the path's type T and in FP64.
template <typename T>
__global__ void twiddle_kernel(C2<T>* tw, C2<double>* tw64, int L) {
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < L; m += gridDim.x * blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * m / L, &sn, &cs);
        tw[m] = cmk(T(cs), T(sn));
        tw64[m] = cmk(cs, sn);
    }
}

struct Layout {
    size_t partial, res, tw[3], tw64[3], vh, sa, sb, dx, table, delta, fac, total;
};

template <typename T>
Layout layout_of(const Dims& dm, int d, bool compressible, bool continuity) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += up256(bytes);
        return at;
    };
    L.partial = take(sizeof(double) * 64 * 1024);
    L.res = take(sizeof(double) * 64);
    for (int a = 0; a < 3; ++a) {
        const int n = a >= 3 - d ? dm.n[a] : 0;
        L.tw[a] = take(sizeof(C2<T>) * n);
        L.tw64[a] = take(sizeof(C2<double>) * n);
    }
    L.vh = take(sizeof(C2<double>) * (size_t)dm.NH * d);
    L.sa = take(sizeof(T) * (size_t)dm.N);
    L.sb = take(sizeof(T) * (size_t)dm.N);
    L.dx = take(sizeof(T) * (size_t)dm.N * d);
    L.table = take(sizeof(int) * (size_t)window_table_ints<T>(dm));
    // the divergence enters the objective only through the continuity
    // state's source factor
    L.delta = continuity && compressible ? take(sizeof(T) * (size_t)dm.N) : 0;
    L.fac = continuity && compressible ? take(sizeof(T) * (size_t)dm.N) : 0;
    L.total = off;
    return L;
}

struct Fail {
    int code;
    std::string msg;
};

#define NACHK(expr)                                                                       \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) throw Fail{GANMRES_EDEVICE, std::string(#expr) + ": " +     \
                                                              hipGetErrorString(e_)};     \
    } while (0)

unsigned char* scratch_base() {
    int dev = 0;
    NACHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Fail{GANMRES_EDEVICE, "device index out of range"};
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        NACHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_ptr[dev] = p;
    }
    return static_cast<unsigned char*>(g_ptr[dev]);
}

template <typename T>
void objective(const ganmres_config& c, const void* m0v, const void* m1v, const void* vv,
               hipStream_t st, double* J, double* mismatch) {
    const int d = c.dim;
    Dims dm{};
    dm.dim = d;
    dm.n[0] = d == 3 ? c.n[0] : 1;
    dm.n[1] = d == 3 ? c.n[1] : c.n[0];
    dm.n[2] = d == 3 ? c.n[2] : c.n[1];
    dm.N = (long long)dm.n[0] * dm.n[1] * dm.n[2];
    dm.n2h = dm.n[2] / 2 + 1;
    dm.NH = (long long)dm.n[0] * dm.n[1] * dm.n2h;
    const bool compressible = !c.incompressible;
    const bool continuity = c.model == GANMRES_CONTINUITY;
    const Layout L = layout_of<T>(dm, d, compressible, continuity);
    if (L.total > kScratchBytes)
        throw Fail{GANMRES_EINVAL, "problem needs " + std::to_string(L.total) +
                                       " bytes of scratch; the allocation-free objective holds " +
                                       std::to_string(kScratchBytes)};
    unsigned char* base = scratch_base();
    double* partial = reinterpret_cast<double*>(base + L.partial);
    double* res = reinterpret_cast<double*>(base + L.res);
    SpectralPlans<T> plans{};
    SpectralPlans<double> plans64{};
    double h[3], cscale[3];
    double cell = 1.0;
    for (int a = 0; a < 3; ++a) {
        h[a] = 2.0 * M_PI / dm.n[a];
        if (a >= 3 - d) cell *= h[a];
    }
    const double ht = 1.0 / c.nt;
    for (int cc = 0; cc < d; ++cc) cscale[cc] = ht / h[comp_axis(d, cc)];
    for (int a = 3 - d; a < 3; ++a) {
        C2<T>* tw = reinterpret_cast<C2<T>*>(base + L.tw[a]);
        C2<double>* tw64 = reinterpret_cast<C2<double>*>(base + L.tw64[a]);
        const int n = dm.n[a];
        twiddle_kernel<T><<<(n + 255) / 256, 256, 0, st>>>(tw, tw64, n);
        NACHK(hipGetLastError());
        plans.p[a].L = plans64.p[a].L = n;
        plans.p[a].nrad = make_radices(n, plans.p[a].rad);
        plans64.p[a].nrad = plans.p[a].nrad;
        for (int r = 0; r < kMaxRadices; ++r) plans64.p[a].rad[r] = plans.p[a].rad[r];
        plans.p[a].tw = tw;
        plans64.p[a].tw = tw64;
    }
    const T* v = static_cast<const T*>(vv);
    const T* m0 = static_cast<const T*>(m0v);
    const T* m1 = static_cast<const T*>(m1v);
    // max |u|: picks the gather variants (the host waits for it)
    NACHK(launch_velocity_max<T>(dm, v, cscale, partial, res + 0, st));
    double um = 0.0;
    NACHK(hipMemcpyAsync(&um, res + 0, sizeof(double), hipMemcpyDeviceToHost, st));
    NACHK(hipStreamSynchronize(st));
    const int ubound = spread_bound(um * (1.0 + 1e-6));
    const int dbound = displacement_bound(um, d);
    // R(v) from the FP64 spectrum of v
    C2<double>* vh[3] = {nullptr, nullptr, nullptr};
    const T* vin[3] = {nullptr, nullptr, nullptr};
    for (int cc = 0; cc < d; ++cc) {
        vh[cc] = reinterpret_cast<C2<double>*>(base + L.vh) + cc * dm.NH;
        vin[cc] = v + cc * dm.N;
    }
    NACHK((launch_rfft<T, double>(dm, plans64, vin, vh, d, st)));
    SpecOpParams sp{};
    sp.dim = d;
    sp.p = c.reg_order;
    sp.alpha = c.alpha;
    sp.leray = 0;
    sp.alpha_seg = nullptr;
    NACHK(launch_spec_regvalue<double>(dm, sp, vh, partial, res + 1, st));
    // divergence, departure points, source factor
    T* delta = (compressible && continuity) ? reinterpret_cast<T*>(base + L.delta) : nullptr;
    T* fac = (compressible && continuity) ? reinterpret_cast<T*>(base + L.fac) : nullptr;
    T* dX = reinterpret_cast<T*>(base + L.dx);
    int* table = reinterpret_cast<int*>(base + L.table);
    int table_write = 1;  // the first gather over dX records the windows
    if (delta) {
        const double one = 1.0;
        for (int cc = 0; cc < d; ++cc) {
            const T* f = v + cc * dm.N;
            NACHK(launch_deriv_axis<T>(dm, plans, comp_axis(d, cc), &f, nullptr, &one, 1, cc > 0,
                                       delta, st));
        }
    }
    NACHK(launch_characteristics<T>(dm, v, cscale, ubound, dX, nullptr, st));
    if (fac) {
        NACHK(launch_source_factor<T>(dm, delta, dX, ht, -1.0, dbound, fac, st, table, table_write));
        table_write = 0;
    }
    // n_t semi-Lagrangian steps between the two state fields
    T* sa = reinterpret_cast<T*>(base + L.sa);
    T* sb = reinterpret_cast<T*>(base + L.sb);
    const T* src = m0;
    for (int j = 0; j < c.nt; ++j) {
        T* out = (j % 2 == 0) ? sa : sb;
        NACHK(launch_sl_step<T>(dm, src, dX, fac, dbound, out, st, table, table_write));
        table_write = 0;
        src = out;
    }
    const Seg g{1, 1, dm.N, dm.N};
    NACHK(launch_sumsq_diff<T>(src, m1, nullptr, g, partial, res + 2, st));
    double host[3] = {0.0, 0.0, 0.0};
    NACHK(hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, st));
    NACHK(hipStreamSynchronize(st));
    const double mis = 0.5 * cell * host[2];
    const double reg = cell / double(dm.N) * host[1];
    *J = mis + 0.5 * c.alpha * reg;
    if (mismatch) *mismatch = mis;
}

}  // namespace
}  // namespace gan

extern "C" {

int ganmres_eval_objective_noalloc(const ganmres_config* cfg, const void* m0, const void* m1,
                                   const void* v, void* stream, double* J, double* mismatch) {
    using namespace gan;
    if (!cfg || !m0 || !m1 || !v || !J) {
        handle_free_error() = "null argument";
        return GANMRES_EINVAL;
    }
    std::string why = config_error(*cfg);
    if (why.empty() && cfg->checkpoint_every != 1) why = "no state history is kept: checkpoint_every must be 1";
    if (!why.empty()) {
        handle_free_error() = why;
        return GANMRES_EINVAL;
    }
    try {
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (cfg->dtype == GANMRES_F32) objective<float>(*cfg, m0, m1, v, st, J, mismatch);
        else objective<double>(*cfg, m0, m1, v, st, J, mismatch);
    } catch (const Fail& f) {
        handle_free_error() = f.msg;
        return f.code;
    }
    if (!std::isfinite(*J)) {
        handle_free_error() = "non-finite objective";
        return GANMRES_ENONFINITE;
    }
    handle_free_error().clear();
    return GANMRES_OK;
}

}  // extern "C"
