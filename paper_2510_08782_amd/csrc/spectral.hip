// Fourier pseudo-spectral kernels (Sec. 2.2 of the paper).
//
// All transforms are done one axis at a time on tiles of pencils held in
// LDS (fft_core.hpp).  Two real pencils always travel as one complex pencil
// z = a + i b:
//   * the spectral derivative i k~ is a real operator (k~ odd in k, Nyquist
//     zeroed), so D(a + i b) = D a + i D b and one complex FFT pair yields
//     two real derivatives with no unpacking;
//   * the real-to-half-spectrum transform of the contiguous axis splits
//     Z = FFT(a + i b) into A(k) = (Z(k) + conj Z(L-k)) / 2 and
//     B(k) = (Z(k) - conj Z(L-k)) / (2i), k = 0..L/2.
// A d-dimensional derivative d/dx_j only needs transforms along axis j (the
// d-D Fourier multiplier i k~_j factorises), which is what the body-force
// kernel exploits: one LDS pass per axis and time point, no full 3-D FFT.
// Full transforms (half spectrum (n0, n1, n2/2+1)) serve the regulariser,
// its inverse and the Leray projection.
#include "fft_core.hpp"
#include "launch.hpp"
#include "reduce.hpp"

namespace gan {

// Dynamic LDS of the transform kernels (16-byte aligned for complex<double>).
extern __shared__ double2 gan_smem[];

namespace {

constexpr int kFftThreads = 256;
constexpr int kMaxItems = 16;       // tile elements per thread (2 PC L <= 4096)
constexpr int kMaxTime = 65;

// log2 of the number of complex pencils per tile for pencils of length L.
// Real-pencil tiles hold 2 PC L <= kFftThreads * kMaxItems elements.
int pc_shift_for(int L, int bytes_per_complex, int max_pencils) {
    int s = 0;
    while ((2 << (s + 1)) * L <= kFftThreads * kMaxItems && (2 << s) < max_pencils &&
           (1 << (s + 1)) * L * bytes_per_complex * 2 <= 64 * 1024 && s < 5)
        ++s;
    return s;
}

// log2 of the number of complex pencils per tile of the in-place complex
// transforms (no per-thread accumulators): two LDS buffers within 64 KB.
int pc_shift_c2c(int L, int bytes_per_complex, int ncols) {
    int s = 0;
    while ((2 << s) <= ncols && (2 << s) * L * bytes_per_complex * 2 <= 64 * 1024 && s < 5) ++s;
    return s;
}

// Geometry of a tile of real pencils along `axis`.
struct RealTile {
    long long base;  // element offset of pencil 0, position 0
    int pstride;     // between pencils of the tile
    int estride;     // between positions along the pencil
    int valid;       // pencils of the tile inside the array
};

__device__ inline RealTile real_tile(const Dims& dm, int axis, int npen, int t) {
    RealTile rt;
    const int n0 = dm.n[0], n1 = dm.n[1], n2 = dm.n[2];
    if (axis == 2) {
        const long long q0 = (long long)t * npen;
        const long long rows = (long long)n0 * n1;
        rt.base = q0 * n2;
        rt.pstride = n2;
        rt.estride = 1;
        rt.valid = (int)((rows - q0) < npen ? (rows - q0) : npen);
    } else {
        const int nch = (n2 + npen - 1) / npen;
        const int outer = t / nch, ch = t % nch;
        rt.base = (axis == 1 ? (long long)outer * n1 * n2 : (long long)outer * n2) +
                  (long long)ch * npen;
        rt.pstride = 1;
        rt.estride = axis == 1 ? n2 : n1 * n2;
        rt.valid = (n2 - ch * npen) < npen ? (n2 - ch * npen) : npen;
    }
    return rt;
}

// Element q of a real tile (2 PC pencils x L): pencil r and position i.
__device__ inline void tile_item(const RealTile& rt, int q, int L, int pcshift, int& r, int& i) {
    if (rt.pstride == 1) {
        r = q & ((2 << pcshift) - 1);
        i = q >> (pcshift + 1);
    } else {
        r = q / L;
        i = q - r * L;
    }
}

template <typename T>
struct DerivArgs {
    Dims dm;
    FftPlan<T> pl;
    int axis, pcshift;
    const T* F;
    long long fstride;
    const T* G;
    long long gstride;
    int ntime;
    int accumulate;
    T* out;
    double w[kMaxTime];
};

// out = [out +] sum_t w_t G_t d/dx_axis F_t over one tile of 2 PC real pencils.
template <typename T>
__global__ void __launch_bounds__(kFftThreads) deriv_axis_kernel(DerivArgs<T> a) {
    C2<T>* bufA = reinterpret_cast<C2<T>*>(gan_smem);
    const int L = a.pl.L;
    const int PC = 1 << a.pcshift;
    C2<T>* bufB = bufA + PC * L;
    const RealTile rt = real_tile(a.dm, a.axis, 2 * PC, blockIdx.x);
    const int nitems = 2 * PC * L;
    const T inv_l = T(1) / T(L);

    T acc[kMaxItems];
    long long addr[kMaxItems];
    bool ok[kMaxItems];
#pragma unroll
    for (int e = 0; e < kMaxItems; ++e) {
        const int q = threadIdx.x + e * kFftThreads;
        int r = 0, i = 0;
        if (q < nitems) tile_item(rt, q, L, a.pcshift, r, i);
        ok[e] = q < nitems && r < rt.valid;
        addr[e] = rt.base + (long long)r * rt.pstride + (long long)i * rt.estride;
        acc[e] = (ok[e] && a.accumulate) ? a.out[addr[e]] : T(0);
    }
    for (int t = 0; t < a.ntime; ++t) {
        const T* F = a.F + t * a.fstride;
#pragma unroll
        for (int e = 0; e < kMaxItems; ++e) {
            const int q = threadIdx.x + e * kFftThreads;
            if (q >= nitems) break;
            int r, i;
            tile_item(rt, q, L, a.pcshift, r, i);
            const T val = ok[e] ? F[addr[e]] : T(0);
            T* slot = reinterpret_cast<T*>(&bufA[(i << a.pcshift) + (r & (PC - 1))]);
            slot[r >> a.pcshift] = val;
        }
        __syncthreads();
        C2<T>* X = block_fft<T>(bufA, bufB, a.pl, a.pcshift, -1);
        for (int q = threadIdx.x; q < PC * L; q += kFftThreads) {
            const int i = q >> a.pcshift;
            X[q] = cmuli(X[q], T(wavenumber_odd(i, L)) * inv_l);
        }
        __syncthreads();
        C2<T>* Y = block_fft<T>(X, X == bufA ? bufB : bufA, a.pl, a.pcshift, +1);
        const T* G = a.G ? a.G + t * a.gstride : nullptr;
        const T wt = T(a.w[t]);
#pragma unroll
        for (int e = 0; e < kMaxItems; ++e) {
            const int q = threadIdx.x + e * kFftThreads;
            if (q >= nitems) break;
            int r, i;
            tile_item(rt, q, L, a.pcshift, r, i);
            const C2<T> z = Y[(i << a.pcshift) + (r & (PC - 1))];
            const T d = (r >> a.pcshift) ? z.y : z.x;
            if (ok[e]) acc[e] += wt * (G ? G[addr[e]] : T(1)) * d;
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < kMaxItems; ++e)
        if (ok[e]) a.out[addr[e]] = acc[e];
}

template <typename T>
struct SpecPtrs {
    C2<T>* spec[3];
};
template <typename T>
struct InPtrs {
    const T* in[3];
};
template <typename T>
struct OutPtrs {
    T* out[3];
    const T* add[3];
};

// Real rows (axis 2) of type TI -> half-spectrum rows computed and stored in
// precision TC, for field blockIdx.y.
template <typename TI, typename TC>
__global__ void __launch_bounds__(kFftThreads) r2c_rows_kernel(Dims dm, FftPlan<TC> pl, int pcshift,
                                                               InPtrs<TI> ip, SpecPtrs<TC> sp) {
    using T = TC;
    C2<T>* bufA = reinterpret_cast<C2<T>*>(gan_smem);
    const int L = pl.L;
    const int PC = 1 << pcshift;
    C2<T>* bufB = bufA + PC * L;
    const TI* in = ip.in[blockIdx.y];
    C2<T>* spec = sp.spec[blockIdx.y];
    const RealTile rt = real_tile(dm, 2, 2 * PC, blockIdx.x);
    const long long q0 = (long long)blockIdx.x * 2 * PC;
    for (int q = threadIdx.x; q < 2 * PC * L; q += kFftThreads) {
        const int r = q / L, i = q - r * L;
        const T val = r < rt.valid ? T(in[rt.base + (long long)r * L + i]) : T(0);
        T* slot = reinterpret_cast<T*>(&bufA[(i << pcshift) + (r & (PC - 1))]);
        slot[r >> pcshift] = val;
    }
    __syncthreads();
    const C2<T>* Z = block_fft<T>(bufA, bufB, pl, pcshift, -1);
    const int nh = dm.n2h;
    for (int q = threadIdx.x; q < 2 * PC * nh; q += kFftThreads) {
        const int r = q / nh, k = q - r * nh;
        if (r >= rt.valid) continue;
        const int p = r & (PC - 1);
        const C2<T> zk = Z[(k << pcshift) + p];
        const int km = k == 0 ? 0 : L - k;
        const C2<T> zm = Z[(km << pcshift) + p];
        C2<T> o;
        if ((r >> pcshift) == 0) o = cmk(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));
        else o = cmk(T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x));
        spec[(q0 + r) * nh + k] = o;
    }
}

// In-place complex transform of the half spectrum along axis 0 or 1.
template <typename T>
__global__ void __launch_bounds__(kFftThreads) c2c_axis_kernel(Dims dm, FftPlan<T> pl, int axis,
                                                               int pcshift, int dir,
                                                               SpecPtrs<T> sp) {
    C2<T>* bufA = reinterpret_cast<C2<T>*>(gan_smem);
    const int L = pl.L;
    const int PC = 1 << pcshift;
    C2<T>* bufB = bufA + PC * L;
    C2<T>* spec = sp.spec[blockIdx.y];
    const int nh = dm.n2h;
    const int nch = (nh + PC - 1) / PC;
    const int outer = blockIdx.x / nch, ch = blockIdx.x % nch;
    const long long base = (axis == 1 ? (long long)outer * dm.n[1] * nh : (long long)outer * nh) +
                           (long long)ch * PC;
    const long long es = axis == 1 ? nh : (long long)dm.n[1] * nh;
    const int valid = (nh - ch * PC) < PC ? (nh - ch * PC) : PC;
    for (int q = threadIdx.x; q < PC * L; q += kFftThreads) {
        const int p = q & (PC - 1), i = q >> pcshift;
        bufA[q] = p < valid ? spec[base + p + i * es] : cmk(T(0), T(0));
    }
    __syncthreads();
    const C2<T>* Z = block_fft<T>(bufA, bufB, pl, pcshift, dir);
    for (int q = threadIdx.x; q < PC * L; q += kFftThreads) {
        const int p = q & (PC - 1), i = q >> pcshift;
        if (p < valid) spec[base + p + i * es] = Z[q];
    }
}

// Half-spectrum rows -> real rows: out = scale * x [+ add].
template <typename T>
__global__ void __launch_bounds__(kFftThreads) c2r_rows_kernel(Dims dm, FftPlan<T> pl, int pcshift,
                                                               T scale, SpecPtrs<T> sp,
                                                               OutPtrs<T> op) {
    C2<T>* bufA = reinterpret_cast<C2<T>*>(gan_smem);
    const int L = pl.L;
    const int PC = 1 << pcshift;
    C2<T>* bufB = bufA + PC * L;
    const C2<T>* spec = sp.spec[blockIdx.y];
    T* out = op.out[blockIdx.y];
    const T* add = op.add[blockIdx.y];
    const RealTile rt = real_tile(dm, 2, 2 * PC, blockIdx.x);
    const long long q0 = (long long)blockIdx.x * 2 * PC;
    const int nh = dm.n2h;
    for (int q = threadIdx.x; q < PC * L; q += kFftThreads) {
        const int p = q / L, i = q - p * L;
        const bool upper = 2 * i > L;
        const int ks = upper ? L - i : i;
        C2<T> A = cmk(T(0), T(0)), B = cmk(T(0), T(0));
        if (p < rt.valid) A = spec[(q0 + p) * nh + ks];
        if (p + PC < rt.valid) B = spec[(q0 + p + PC) * nh + ks];
        if (ks == 0 || 2 * ks == L) {
            A.y = T(0);
            B.y = T(0);
        }
        if (upper) {
            A.y = -A.y;
            B.y = -B.y;
        }
        bufA[(i << pcshift) + p] = cmk(A.x - B.y, A.y + B.x);
    }
    __syncthreads();
    const C2<T>* Z = block_fft<T>(bufA, bufB, pl, pcshift, +1);
    for (int q = threadIdx.x; q < 2 * PC * L; q += kFftThreads) {
        const int r = q / L, i = q - r * L;
        if (r >= rt.valid) continue;
        const C2<T> z = Z[(i << pcshift) + (r & (PC - 1))];
        const long long o = rt.base + (long long)r * L + i;
        T val = scale * ((r >> pcshift) ? z.y : z.x);
        if (add) val += add[o];
        out[o] = val;
    }
}

// ---- pointwise operators on the half spectrum --------------------------------
struct KVec {
    double k2;       // |k|^2 (Nyquist kept)
    double kt[3];    // k~ per internal axis (Nyquist zeroed)
};

__device__ inline KVec kvec(const Dims& dm, long long lin) {
    const int nh = dm.n2h;
    const int i2 = (int)(lin % nh);
    const long long rest = lin / nh;
    const int i1 = (int)(rest % dm.n[1]);
    const int i0 = (int)(rest / dm.n[1]);
    KVec kv;
    const int k0 = wavenumber(i0, dm.n[0]), k1 = wavenumber(i1, dm.n[1]), k2 = i2;
    kv.k2 = double(k0) * k0 + double(k1) * k1 + double(k2) * k2;
    kv.kt[0] = wavenumber_odd(i0, dm.n[0]);
    kv.kt[1] = wavenumber_odd(i1, dm.n[1]);
    kv.kt[2] = (2 * i2 == dm.n[2]) ? 0.0 : double(i2);
    return kv;
}

__device__ inline double ipow(double x, int p) {
    double r = x;
    for (int i = 1; i < p; ++i) r *= x;
    return r;
}

// Leray projection of the d components (in place on u).
template <typename T>
__device__ inline void leray_point(const KVec& kv, int dim, C2<T>* u) {
    double kk = 0.0;
    double kc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        kc[c] = c < dim ? kv.kt[comp_axis(dim, c)] : 0.0;
        kk += kc[c] * kc[c];
    }
    if (kk == 0.0) return;
    C2<T> dot = cmk(T(0), T(0));
#pragma unroll
    for (int c = 0; c < 3; ++c) dot = cadd(dot, cscale(u[c], T(kc[c])));
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = csub(u[c], cscale(dot, T(kc[c] / kk)));
}

// The regulariser term is formed from an FP64 spectrum of v: l_p(k) grows like
// |k|^(2p), so rounding noise of an FP32 transform in the high modes would be
// amplified into the gradient.
template <typename T>
__global__ void spec_gradient_kernel(Dims dm, SpecOpParams sp, SpecPtrs<double> vh, SpecPtrs<T> bh,
                                     SpecPtrs<T> gh) {
    for (long long lin = blockIdx.x * (long long)blockDim.x + threadIdx.x; lin < dm.NH;
         lin += (long long)gridDim.x * blockDim.x) {
        const KVec kv = kvec(dm, lin);
        const double al = sp.alpha * ipow(kv.k2, sp.p);
        C2<T> b[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) b[c] = c < sp.dim ? bh.spec[c][lin] : cmk(T(0), T(0));
        if (sp.leray) leray_point(kv, sp.dim, b);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (c < sp.dim) {
                const C2<double> z = vh.spec[c][lin];
                gh.spec[c][lin] = cmk(T(al * z.x + double(b[c].x)), T(al * z.y + double(b[c].y)));
            }
    }
}

template <typename T>
__global__ void spec_precond_kernel(Dims dm, SpecOpParams sp, SpecPtrs<T> gh, SpecPtrs<T> sh) {
    for (long long lin = blockIdx.x * (long long)blockDim.x + threadIdx.x; lin < dm.NH;
         lin += (long long)gridDim.x * blockDim.x) {
        const KVec kv = kvec(dm, lin);
        double l = ipow(kv.k2, sp.p);
        if (l == 0.0) l = 1.0;
        const T f = T(-1.0 / (sp.alpha * l));
        C2<T> g[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) g[c] = c < sp.dim ? gh.spec[c][lin] : cmk(T(0), T(0));
        if (sp.leray) leray_point(kv, sp.dim, g);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (c < sp.dim) sh.spec[c][lin] = cscale(g[c], f);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) spec_regvalue_kernel(Dims dm, SpecOpParams sp,
                                                            SpecPtrs<T> vh, double* partial) {
    __shared__ double sh[256 / 64];
    double acc = 0.0;
    for (long long lin = blockIdx.x * (long long)blockDim.x + threadIdx.x; lin < dm.NH;
         lin += (long long)gridDim.x * blockDim.x) {
        const KVec kv = kvec(dm, lin);
        const int i2 = (int)(lin % dm.n2h);
        const double wgt = (i2 == 0 || 2 * i2 == dm.n[2]) ? 1.0 : 2.0;
        const double l = ipow(kv.k2, sp.p);
        double s = 0.0;
        for (int c = 0; c < sp.dim; ++c) {
            const C2<T> z = vh.spec[c][lin];
            s += double(z.x) * double(z.x) + double(z.y) * double(z.y);
        }
        acc += wgt * l * s;
    }
    const double r = block_reduce<false>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

inline int pointwise_blocks(long long n) {
    long long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    return (int)(b < 1 ? 1 : b);
}

template <typename T>
int real_tiles(const Dims& dm, int axis, int npen) {
    if (axis == 2) return (int)(((long long)dm.n[0] * dm.n[1] + npen - 1) / npen);
    const int nch = (dm.n[2] + npen - 1) / npen;
    return (axis == 1 ? dm.n[0] : dm.n[1]) * nch;
}

}  // namespace

template <typename T>
hipError_t launch_deriv_axis(const Dims& dm, const SpectralPlans<T>& pl, int axis, const T* F,
                             long long fstride, const T* G, long long gstride, const double* w,
                             int ntime, int accumulate, T* out, hipStream_t st) {
    if (ntime < 1 || ntime > kMaxTime) return hipErrorInvalidValue;
    DerivArgs<T> a;
    a.dm = dm;
    a.pl = pl.p[axis];
    a.axis = axis;
    const int L = dm.n[axis];
    const int pencils = axis == 2 ? dm.n[0] * dm.n[1] : dm.n[2];
    a.pcshift = pc_shift_for(L, (int)sizeof(C2<T>), pencils);
    a.F = F;
    a.fstride = fstride;
    a.G = G;
    a.gstride = gstride;
    a.ntime = ntime;
    a.accumulate = accumulate;
    a.out = out;
    for (int t = 0; t < kMaxTime; ++t) a.w[t] = t < ntime ? w[t] : 0.0;
    const int PC = 1 << a.pcshift;
    const size_t lds = 2 * (size_t)PC * L * sizeof(C2<T>);
    const int tiles = real_tiles<T>(dm, axis, 2 * PC);
    deriv_axis_kernel<T><<<tiles, kFftThreads, lds, st>>>(a);
    return hipGetLastError();
}

template <typename TI, typename TC>
hipError_t launch_rfft(const Dims& dm, const SpectralPlans<TC>& pl, const TI* const* in,
                       C2<TC>* const* out, int count, hipStream_t st) {
    if (count < 1 || count > 3) return hipErrorInvalidValue;
    InPtrs<TI> ip{};
    SpecPtrs<TC> sp{};
    for (int c = 0; c < count; ++c) {
        ip.in[c] = in[c];
        sp.spec[c] = out[c];
    }
    {
        const int L = dm.n[2];
        const int sh = pc_shift_for(L, (int)sizeof(C2<TC>), dm.n[0] * dm.n[1]);
        const int PC = 1 << sh;
        const size_t lds = 2 * (size_t)PC * L * sizeof(C2<TC>);
        dim3 g(real_tiles<TC>(dm, 2, 2 * PC), count);
        r2c_rows_kernel<TI, TC><<<g, kFftThreads, lds, st>>>(dm, pl.p[2], sh, ip, sp);
    }
    for (int axis = 1; axis >= 3 - dm.dim; --axis) {
        const int L = dm.n[axis];
        const int sh = pc_shift_c2c(L, (int)sizeof(C2<TC>), dm.n2h);
        const int PC = 1 << sh;
        const size_t lds = 2 * (size_t)PC * L * sizeof(C2<TC>);
        const int nch = (dm.n2h + PC - 1) / PC;
        dim3 g((axis == 1 ? dm.n[0] : dm.n[1]) * nch, count);
        c2c_axis_kernel<TC><<<g, kFftThreads, lds, st>>>(dm, pl.p[axis], axis, sh, -1, sp);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_irfft(const Dims& dm, const SpectralPlans<T>& pl, C2<T>* const* spec,
                        T* const* out, const T* const* add, double scale, int count,
                        hipStream_t st) {
    if (count < 1 || count > 3) return hipErrorInvalidValue;
    SpecPtrs<T> sp{};
    OutPtrs<T> op{};
    for (int c = 0; c < count; ++c) {
        sp.spec[c] = spec[c];
        op.out[c] = out[c];
        op.add[c] = add ? add[c] : nullptr;
    }
    for (int axis = 3 - dm.dim; axis <= 1; ++axis) {
        const int L = dm.n[axis];
        const int sh = pc_shift_c2c(L, (int)sizeof(C2<T>), dm.n2h);
        const int PC = 1 << sh;
        const size_t lds = 2 * (size_t)PC * L * sizeof(C2<T>);
        const int nch = (dm.n2h + PC - 1) / PC;
        dim3 g((axis == 1 ? dm.n[0] : dm.n[1]) * nch, count);
        c2c_axis_kernel<T><<<g, kFftThreads, lds, st>>>(dm, pl.p[axis], axis, sh, +1, sp);
    }
    {
        const int L = dm.n[2];
        const int sh = pc_shift_for(L, (int)sizeof(C2<T>), dm.n[0] * dm.n[1]);
        const int PC = 1 << sh;
        const size_t lds = 2 * (size_t)PC * L * sizeof(C2<T>);
        dim3 g(real_tiles<T>(dm, 2, 2 * PC), count);
        c2r_rows_kernel<T><<<g, kFftThreads, lds, st>>>(dm, pl.p[2], sh, T(scale), sp, op);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_gradient(const Dims& dm, const SpecOpParams& sp, C2<double>* const* vh,
                                C2<T>* const* bh, C2<T>* const* gh, hipStream_t st) {
    SpecPtrs<double> a{};
    SpecPtrs<T> b{}, g{};
    for (int c = 0; c < sp.dim; ++c) {
        a.spec[c] = vh[c];
        b.spec[c] = bh[c];
        g.spec[c] = gh[c];
    }
    spec_gradient_kernel<T><<<pointwise_blocks(dm.NH), 256, 0, st>>>(dm, sp, a, b, g);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_precond(const Dims& dm, const SpecOpParams& sp, C2<T>* const* gh,
                               C2<T>* const* sh, hipStream_t st) {
    SpecPtrs<T> a{}, b{};
    for (int c = 0; c < sp.dim; ++c) {
        a.spec[c] = gh[c];
        b.spec[c] = sh[c];
    }
    spec_precond_kernel<T><<<pointwise_blocks(dm.NH), 256, 0, st>>>(dm, sp, a, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_regvalue(const Dims& dm, const SpecOpParams& sp, C2<T>* const* vh,
                                double* partial, double* res, hipStream_t st) {
    SpecPtrs<T> a{};
    for (int c = 0; c < sp.dim; ++c) a.spec[c] = vh[c];
    const int nb = reduction_blocks(dm.NH);
    spec_regvalue_kernel<T><<<nb, 256, 0, st>>>(dm, sp, a, partial);
    finish_kernel<false><<<1, 1024, 0, st>>>(partial, nb, 1, res);
    return hipGetLastError();
}

#define GAN_INST(T)                                                                               \
    template hipError_t launch_deriv_axis<T>(const Dims&, const SpectralPlans<T>&, int, const T*, \
                                             long long, const T*, long long, const double*, int,  \
                                             int, T*, hipStream_t);                               \
    template hipError_t launch_rfft<T, T>(const Dims&, const SpectralPlans<T>&, const T* const*,  \
                                          C2<T>* const*, int, hipStream_t);                       \
    template hipError_t launch_irfft<T>(const Dims&, const SpectralPlans<T>&, C2<T>* const*,      \
                                        T* const*, const T* const*, double, int, hipStream_t);    \
    template hipError_t launch_spec_gradient<T>(const Dims&, const SpecOpParams&,                 \
                                                C2<double>* const*, C2<T>* const*, C2<T>* const*, \
                                                hipStream_t);                                     \
    template hipError_t launch_spec_precond<T>(const Dims&, const SpecOpParams&, C2<T>* const*,   \
                                               C2<T>* const*, hipStream_t);                       \
    template hipError_t launch_spec_regvalue<T>(const Dims&, const SpecOpParams&, C2<T>* const*,  \
                                                double*, double*, hipStream_t);
GAN_INST(float)
GAN_INST(double)
#undef GAN_INST
template hipError_t launch_rfft<float, double>(const Dims&, const SpectralPlans<double>&,
                                               const float* const*, C2<double>* const*, int,
                                               hipStream_t);

}  // namespace gan
