// Semi-Lagrangian kernels: RK2 characteristics, the cubic Lagrange gather
// step of the state / adjoint solves, and the stationary source factors.
//
// Paper, Sec. 2.2: semi-Lagrangian time integration with an explicit RK2
// backtrace.  The interpolation at departure points is the tensor-product
// cubic Lagrange stencil (4 taps per axis: nodes f-1..f+2 around
// f = floor(xi)), periodic in every axis.  Departure points are stored as
// displacements in cells, so the fractional offset t keeps full precision in
// FP32 whatever the grid index.
//
// LDS-tiled gather.  A block owns a tile of output points (3-D: 32 x 8 x TZ,
// 2-D: 64 x 32) and stages the source field over the tile plus a fixed halo
// of HALO+1 cells below and HALO+2 above every axis, loaded row by row with
// coalesced reads.  Every tap then comes from LDS at a compile-time offset
// from one base address per point.  The halo covers departure displacements
// up to HALO cells; the bound of the current displacement field is computed
// on the device (ceil of max |d|, one int per field) and read by the kernel,
// which switches the whole launch to a direct global gather when the bound
// exceeds HALO (large line-search trial steps).  The fallback gives the same
// values: only where the taps are read from changes.
#include "launch.hpp"
#include "reduce.hpp"

namespace gan {

namespace {

constexpr int kThreads = 256;

template <typename T>
__device__ inline void lagrange4(T t, T* w) {
    const T tp1 = t + T(1), tm1 = t - T(1), tm2 = t - T(2);
    const T sixth = T(1.0 / 6.0);
    w[0] = -t * tm1 * tm2 * sixth;
    w[1] = tp1 * tm1 * tm2 * T(0.5);
    w[2] = -tp1 * t * tm2 * T(0.5);
    w[3] = tp1 * t * tm1 * sixth;
}

template <typename T>
__device__ inline T clamp_disp(T d) {
    return fmin(fmax(d, T(-1.0e7)), T(1.0e7));
}

// Taps along one axis for a global gather: element offsets (times the axis
// stride) and weights for displacement `disp` from grid index i.
template <typename T>
__device__ inline void axis_taps(int i, T disp, int n, int stride, int* off, T* w) {
    disp = clamp_disp(disp);
    const T fl = floor(disp);
    lagrange4(disp - fl, w);
    const int b = pmod(i + static_cast<int>(fl), n);
    const int bm = (b == 0) ? n - 1 : b - 1;
    const int b1 = (b + 1 == n) ? 0 : b + 1;
    const int b2 = (b1 + 1 == n) ? 0 : b1 + 1;
    off[0] = bm * stride;
    off[1] = b * stride;
    off[2] = b1 * stride;
    off[3] = b2 * stride;
}

// Direct (L1/L2) gather of one field at point (i0,i1,i2) + (d0,d1,d2).
template <typename T, int DIM>
__device__ inline T gather_global(const Dims& dm, const T* __restrict__ s, int i0, int i1, int i2,
                                  T d0, T d1, T d2) {
    int o1[4], o2[4];
    T w1[4], w2[4];
    axis_taps(i1, d1, dm.n[1], dm.n[2], o1, w1);
    axis_taps(i2, d2, dm.n[2], 1, o2, w2);
    T acc = T(0);
    if constexpr (DIM == 3) {
        int o0[4];
        T w0[4];
        axis_taps(i0, d0, dm.n[0], dm.n[1] * dm.n[2], o0, w0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            T sa = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const T* row = s + o0[a] + o1[b];
                sa += w1[b] * (w2[0] * row[o2[0]] + w2[1] * row[o2[1]] + w2[2] * row[o2[2]] +
                               w2[3] * row[o2[3]]);
            }
            acc += w0[a] * sa;
        }
    } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T* row = s + o1[b];
            acc += w1[b] * (w2[0] * row[o2[0]] + w2[1] * row[o2[1]] + w2[2] * row[o2[2]] +
                            w2[3] * row[o2[3]]);
        }
    }
    return acc;
}

// ---- tile geometry -----------------------------------------------------------
// 3-D: threads (32 x 8), each owns TZ points along z.  2-D: threads (64 x 4),
// each owns 8 points along y (tile 64 x 32).
template <typename T, int DIM>
struct Tile;
#ifndef GAN_SL_TZ32
#define GAN_SL_TZ32 8
#endif
#ifndef GAN_SL_HALO3
#define GAN_SL_HALO3 2
#endif
#ifndef GAN_SL_TX3
#define GAN_SL_TX3 32
#endif
template <typename T>
struct Tile<T, 3> {
    static constexpr int TX = GAN_SL_TX3, TY = 256 / GAN_SL_TX3, TZ = sizeof(T) == 4 ? GAN_SL_TZ32 : 4;
    static constexpr int HALO = GAN_SL_HALO3;
    static constexpr int RX = TX + 2 * HALO + 3, RY = TY + 2 * HALO + 3, RZ = TZ + 2 * HALO + 3;
    static constexpr int PTS = TZ;  // points per thread
};
template <typename T>
struct Tile<T, 2> {
    static constexpr int TX = 64, TY = 32, TZ = 1;
    static constexpr int HALO = 4;
    static constexpr int RX = TX + 2 * HALO + 3, RY = TY + 2 * HALO + 3, RZ = 1;
    static constexpr int PTS = 8;
};

template <typename T, int DIM>
constexpr size_t tile_lds_bytes() {
    using C = Tile<T, DIM>;
    return sizeof(T) * C::RX * C::RY * C::RZ;
}

// g mod n in [0, n): the common in-range case costs one compare.
__device__ inline int wrapn(int g, int n) {
    return (static_cast<unsigned>(g) < static_cast<unsigned>(n)) ? g : pmod(g, n);
}

// Stage src over the block's tile + halo (origin x0,y0,z0 of the tile).
// Global-to-LDS loads (global_load_lds_dword): a wavefront walks the rows of
// the region and moves each row with one instruction per 64 dwords, lane l
// writing dword l of the row; the wrapped x index of every lane is computed
// once.  All of a wave's row loads are in flight together and no VGPRs hold
// the data.  FP64 rows move as pairs of dwords.  Ends with a barrier.
template <typename T, int DIM>
__device__ inline void stage(const Dims& dm, const T* __restrict__ src, T* lds, int x0, int y0,
                             int z0) {
    using C = Tile<T, DIM>;
    constexpr int W = sizeof(T) / 4;                  // dwords per element
    constexpr int ROWS = C::RY * C::RZ;
    constexpr int NW = kThreads / 64;
    constexpr int XP = (W * C::RX + 63) / 64;         // dword passes per row
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int goff[XP];                                    // dword offset of the lane's element in a row
    bool xin[XP];
#pragma unroll
    for (int u = 0; u < XP; ++u) {
        const int d = lane + 64 * u;
        xin[u] = d < W * C::RX;
        goff[u] = W * wrapn(x0 - C::HALO - 1 + d / W, dm.n[2]) + d % W;
    }
    for (int r = wave; r < ROWS; r += NW) {
        const int ry = r % C::RY, rz = r / C::RY;
        const int gy = wrapn(y0 - C::HALO - 1 + ry, dm.n[1]);
        const int gz = DIM == 3 ? wrapn(z0 - C::HALO - 1 + rz, dm.n[0]) : 0;
        // N < 2^31 elements
        const unsigned* row = reinterpret_cast<const unsigned*>(src + (gz * dm.n[1] + gy) * dm.n[2]);
        unsigned* dst = reinterpret_cast<unsigned*>(lds + r * C::RX);
#pragma unroll
        for (int u = 0; u < XP; ++u)
            if (xin[u]) __builtin_amdgcn_global_load_lds(row + goff[u], dst + 64 * u, 4, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Tap base and weights along one axis for the LDS path: local index of the
// node f-1 (relative to the region origin) for point index li within the tile.
template <typename T, int HALO, int R>
__device__ inline int lds_axis(int li, T disp, T* w) {
    const T fl = floor(disp);
    lagrange4(disp - fl, w);
    int l = li + static_cast<int>(fl) + HALO;  // = (li + fl + HALO + 1) - 1
    l = l < 0 ? 0 : (l > R - 4 ? R - 4 : l);
    return l;
}

// Interpolate from the staged region at tile-local point (lx,ly,lz) displaced by d.
template <typename T, int DIM>
__device__ inline T gather_lds(const T* lds, int lx, int ly, int lz, T d0, T d1, T d2) {
    using C = Tile<T, DIM>;
    T wx[4], wy[4];
    const int bx = lds_axis<T, C::HALO, C::RX>(lx, d2, wx);
    const int by = lds_axis<T, C::HALO, C::RY>(ly, d1, wy);
    T acc = T(0);
    if constexpr (DIM == 3) {
        T wz[4];
        const int bz = lds_axis<T, C::HALO, C::RZ>(lz, d0, wz);
        const T* base = lds + (bz * C::RY + by) * C::RX + bx;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            T sa = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const T* row = base + (a * C::RY + b) * C::RX;
                sa += wy[b] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2] + wx[3] * row[3]);
            }
            acc += wz[a] * sa;
        }
    } else {
        const T* base = lds + by * C::RX + bx;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T* row = base + b * C::RX;
            acc += wy[b] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2] + wx[3] * row[3]);
        }
    }
    return acc;
}

// Tile origin of this block and the local coordinates of the thread's k-th point.
template <typename T, int DIM>
struct PointMap {
    int x0, y0, z0;
    __device__ PointMap(const Dims& dm) {
        using C = Tile<T, DIM>;
        const int ntx = (dm.n[2] + C::TX - 1) / C::TX;
        const int nty = (dm.n[1] + C::TY - 1) / C::TY;
        const int b = blockIdx.x;
        x0 = (b % ntx) * C::TX;
        y0 = ((b / ntx) % nty) * C::TY;
        z0 = (b / (ntx * nty)) * C::TZ;
    }
    // local (lx, ly, lz) of point k of this thread
    __device__ void local(int k, int& lx, int& ly, int& lz) const {
        if constexpr (DIM == 3) {
            using C = Tile<T, 3>;
            lx = threadIdx.x % C::TX;
            ly = threadIdx.x / C::TX;
            lz = k;
        } else {
            lx = threadIdx.x & 63;
            ly = (threadIdx.x >> 6) + 4 * k;
            lz = 0;
        }
    }
};

template <typename T, int DIM>
int tile_blocks(const Dims& dm) {
    using C = Tile<T, DIM>;
    const int ntx = (dm.n[2] + C::TX - 1) / C::TX;
    const int nty = (dm.n[1] + C::TY - 1) / C::TY;
    const int ntz = DIM == 3 ? (dm.n[0] + C::TZ - 1) / C::TZ : 1;
    return ntx * nty * ntz;
}

// ---- semi-Lagrangian step --------------------------------------------------------
// EPI 0: out = I[src];  1: out = fac * I[src];
// EPI 2 (source factor, src = delta): out = 1 + sgn h/2 (I[d] + d) + h^2/2 d I[d]
template <typename T, int DIM, int EPI>
__global__ void __launch_bounds__(kThreads) sl_step_kernel(Dims dm, const T* __restrict__ src,
                                                           const T* __restrict__ disp,
                                                           const T* __restrict__ fac, T ht, T sgn,
                                                           const int* __restrict__ bound,
                                                           T* __restrict__ out) {
    using C = Tile<T, DIM>;
    extern __shared__ double2 sl_smem[];
    T* lds = reinterpret_cast<T*>(sl_smem);
    const PointMap<T, DIM> pm(dm);
    const bool use_lds = *bound <= C::HALO;
    const long long N = dm.N;
    // displacements of the thread's points, loaded before the staging
    T d0[C::PTS], d1[C::PTS], d2[C::PTS];
    long long lin[C::PTS];
    bool in[C::PTS];
#pragma unroll
    for (int k = 0; k < C::PTS; ++k) {
        int lx, ly, lz;
        pm.local(k, lx, ly, lz);
        const int i2 = pm.x0 + lx, i1 = pm.y0 + ly, i0 = pm.z0 + lz;
        in[k] = i2 < dm.n[2] && i1 < dm.n[1] && i0 < dm.n[0];
        lin[k] = ((long long)i0 * dm.n[1] + i1) * dm.n[2] + i2;
        d0[k] = d1[k] = d2[k] = T(0);
        if (in[k]) {
            if constexpr (DIM == 3) {
                d0[k] = disp[lin[k]];
                d1[k] = disp[N + lin[k]];
                d2[k] = disp[2 * N + lin[k]];
            } else {
                d1[k] = disp[lin[k]];
                d2[k] = disp[N + lin[k]];
            }
        }
    }
    if (use_lds) stage<T, DIM>(dm, src, lds, pm.x0, pm.y0, pm.z0);
#pragma unroll
    for (int k = 0; k < C::PTS; ++k) {
        if (!in[k]) continue;
        int lx, ly, lz;
        pm.local(k, lx, ly, lz);
        T r;
        if (use_lds) {
            r = gather_lds<T, DIM>(lds, lx, ly, lz, d0[k], d1[k], d2[k]);
        } else {
            r = gather_global<T, DIM>(dm, src, pm.z0 + lz, pm.y0 + ly, pm.x0 + lx, d0[k], d1[k],
                                      d2[k]);
        }
        if constexpr (EPI == 1) r *= fac[lin[k]];
        if constexpr (EPI == 2) {
            const T dc = src[lin[k]];
            r = T(1) + sgn * T(0.5) * ht * (r + dc) + T(0.5) * ht * ht * dc * r;
        }
        out[lin[k]] = r;
    }
}

// ---- characteristics -------------------------------------------------------------
// dX = -(u + I[u](i - u)) / 2 (state, +v) and dY = (u + I[u](i + u)) / 2
// (adjoint, -v), u_c = s_c v_c.  Component c of v is staged in LDS in turn;
// the predictor points only depend on u at the grid point.  The ceil of the
// largest |dX| / |dY| is accumulated into bound_out[0] / bound_out[1].
template <typename T, int DIM, bool DOX, bool DOY>
__global__ void __launch_bounds__(kThreads) characteristics_kernel(
    Dims dm, const T* __restrict__ v, T s0, T s1, T s2, const int* __restrict__ ubound,
    T* __restrict__ dX, T* __restrict__ dY, int* __restrict__ bound_out) {
    using C = Tile<T, DIM>;
    extern __shared__ double2 sl_smem[];
    T* lds = reinterpret_cast<T*>(sl_smem);
    __shared__ int smax[2];
    if (threadIdx.x < 2) smax[threadIdx.x] = 0;
    const PointMap<T, DIM> pm(dm);
    const bool use_lds = *ubound <= C::HALO;
    const long long N = dm.N;
    const T s[3] = {s0, s1, s2};
    int mx = 0, my = 0;
    for (int c = 0; c < DIM; ++c) {
        const T* vc = v + c * N;
        if (use_lds) {
            __syncthreads();
            stage<T, DIM>(dm, vc, lds, pm.x0, pm.y0, pm.z0);
        }
#pragma unroll 1
        for (int k = 0; k < C::PTS; ++k) {
            int lx, ly, lz;
            pm.local(k, lx, ly, lz);
            const int i2 = pm.x0 + lx, i1 = pm.y0 + ly, i0 = pm.z0 + lz;
            if (i2 >= dm.n[2] || i1 >= dm.n[1] || i0 >= dm.n[0]) continue;
            const long long lin = ((long long)i0 * dm.n[1] + i1) * dm.n[2] + i2;
            T u[3];
#pragma unroll
            for (int q = 0; q < DIM; ++q) u[q] = v[q * N + lin] * s[q];
            T e0 = T(0), e1, e2;
            if constexpr (DIM == 3) {
                e0 = u[0];
                e1 = u[1];
                e2 = u[2];
            } else {
                e1 = u[0];
                e2 = u[1];
            }
            if (DOX) {
                const T iv = use_lds ? gather_lds<T, DIM>(lds, lx, ly, lz, -e0, -e1, -e2)
                                     : gather_global<T, DIM>(dm, vc, i0, i1, i2, -e0, -e1, -e2);
                const T d = T(-0.5) * (u[c] + s[c] * iv);
                dX[c * N + lin] = d;
                const T ad = fabs(d);
                mx = max(mx, ad <= T(1.0e6) ? static_cast<int>(ceil(ad)) : 1 << 30);
            }
            if (DOY) {
                const T iv = use_lds ? gather_lds<T, DIM>(lds, lx, ly, lz, e0, e1, e2)
                                     : gather_global<T, DIM>(dm, vc, i0, i1, i2, e0, e1, e2);
                const T d = T(0.5) * (u[c] + s[c] * iv);
                dY[c * N + lin] = d;
                const T ad = fabs(d);
                my = max(my, ad <= T(1.0e6) ? static_cast<int>(ceil(ad)) : 1 << 30);
            }
        }
    }
    __syncthreads();
    if (mx) atomicMax(&smax[0], mx);
    if (my) atomicMax(&smax[1], my);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (DOX && smax[0]) atomicMax(&bound_out[0], smax[0]);
        if (DOY && smax[1]) atomicMax(&bound_out[1], smax[1]);
    }
}

// ceil(max_c max_i |s_c v_c(i)|) -> atomicMax into *out (the predictor bound).
template <typename T>
__global__ void __launch_bounds__(kThreads) velocity_bound_kernel(const T* __restrict__ v,
                                                                  long long N, int dim, T s0, T s1,
                                                                  T s2, int* __restrict__ out) {
    __shared__ double sh[kThreads / 64];
    const T s[3] = {s0, s1, s2};
    double m = 0.0;
    for (int c = 0; c < dim; ++c)
        for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
             i += (long long)gridDim.x * blockDim.x) {
            double a = fabs(double(v[c * N + i] * s[c]));
            if (!(a <= 1.0e6)) a = 1.0e6;
            m = fmax(m, a);
        }
    const double r = block_reduce<true>(m, sh);
    if (threadIdx.x == 0) atomicMax(out, static_cast<int>(ceil(r)));
}

__global__ void zero_ints_kernel(int* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

}  // namespace

template <typename T>
hipError_t launch_zero_bounds(int* bounds, int n, hipStream_t st) {
    zero_ints_kernel<<<1, 64, 0, st>>>(bounds, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_velocity_bound(const Dims& dm, const T* v, const double* s, int* out,
                                 hipStream_t st) {
    const int nb = reduction_blocks(dm.N);
    velocity_bound_kernel<T><<<nb, kThreads, 0, st>>>(v, dm.N, dm.dim, T(s[0]), T(s[1]),
                                                      T(dm.dim == 3 ? s[2] : 0.0), out);
    return hipGetLastError();
}

template <typename T, int DIM, bool DOX, bool DOY>
void char_launch(const Dims& dm, const T* v, const double* s, const int* ubound, T* dX, T* dY,
                 int* bound_out, hipStream_t st) {
    characteristics_kernel<T, DIM, DOX, DOY>
        <<<tile_blocks<T, DIM>(dm), kThreads, tile_lds_bytes<T, DIM>(), st>>>(
            dm, v, T(s[0]), T(s[1]), T(DIM == 3 ? s[2] : 0.0), ubound, dX, dY, bound_out);
}

// 3-D: one launch per direction (each stages the components of v again but
// keeps one gather in flight per thread); 2-D: both directions in one launch.
template <typename T>
hipError_t launch_characteristics(const Dims& dm, const T* v, const double* s, const int* ubound,
                                  T* dX, T* dY, int* bound_out, hipStream_t st) {
    if (dm.dim == 3) {
        if (dX) char_launch<T, 3, true, false>(dm, v, s, ubound, dX, dY, bound_out, st);
        if (dY) char_launch<T, 3, false, true>(dm, v, s, ubound, dX, dY, bound_out, st);
    } else {
        if (dX && dY) char_launch<T, 2, true, true>(dm, v, s, ubound, dX, dY, bound_out, st);
        else if (dX) char_launch<T, 2, true, false>(dm, v, s, ubound, dX, dY, bound_out, st);
        else if (dY) char_launch<T, 2, false, true>(dm, v, s, ubound, dX, dY, bound_out, st);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sl_step(const Dims& dm, const T* src, const T* disp, const T* fac,
                          const int* bound, T* out, hipStream_t st) {
    if (dm.dim == 3) {
        const dim3 g(tile_blocks<T, 3>(dm));
        const size_t lds = tile_lds_bytes<T, 3>();
        if (fac) sl_step_kernel<T, 3, 1><<<g, kThreads, lds, st>>>(dm, src, disp, fac, T(0), T(0), bound, out);
        else sl_step_kernel<T, 3, 0><<<g, kThreads, lds, st>>>(dm, src, disp, fac, T(0), T(0), bound, out);
    } else {
        const dim3 g(tile_blocks<T, 2>(dm));
        const size_t lds = tile_lds_bytes<T, 2>();
        if (fac) sl_step_kernel<T, 2, 1><<<g, kThreads, lds, st>>>(dm, src, disp, fac, T(0), T(0), bound, out);
        else sl_step_kernel<T, 2, 0><<<g, kThreads, lds, st>>>(dm, src, disp, fac, T(0), T(0), bound, out);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_source_factor(const Dims& dm, const T* delta, const T* disp, double ht,
                                double sgn, const int* bound, T* out, hipStream_t st) {
    if (dm.dim == 3)
        sl_step_kernel<T, 3, 2><<<tile_blocks<T, 3>(dm), kThreads, tile_lds_bytes<T, 3>(), st>>>(
            dm, delta, disp, nullptr, T(ht), T(sgn), bound, out);
    else
        sl_step_kernel<T, 2, 2><<<tile_blocks<T, 2>(dm), kThreads, tile_lds_bytes<T, 2>(), st>>>(
            dm, delta, disp, nullptr, T(ht), T(sgn), bound, out);
    return hipGetLastError();
}

#define GAN_INST(T)                                                                               \
    template hipError_t launch_zero_bounds<T>(int*, int, hipStream_t);                            \
    template hipError_t launch_velocity_bound<T>(const Dims&, const T*, const double*, int*,      \
                                                 hipStream_t);                                    \
    template hipError_t launch_characteristics<T>(const Dims&, const T*, const double*,           \
                                                  const int*, T*, T*, int*, hipStream_t);         \
    template hipError_t launch_sl_step<T>(const Dims&, const T*, const T*, const T*, const int*,  \
                                          T*, hipStream_t);                                       \
    template hipError_t launch_source_factor<T>(const Dims&, const T*, const T*, double, double,  \
                                                const int*, T*, hipStream_t);
GAN_INST(float)
GAN_INST(double)
#undef GAN_INST

}  // namespace gan
