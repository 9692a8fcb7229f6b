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
// 2-D: 64 x 32) and stages the source field over the tile plus a halo of
// H+1 cells below and H+2 above every axis.  Every tap then comes from LDS at
// a compile-time offset from one base address per point.  The caller passes
// an upper bound on the displacement (cells); the launcher picks the smallest
// halo variant that covers it, and a launch whose bound exceeds its halo takes
// the direct global gather instead.  Both paths give the same values: only
// where the taps are read from changes.
#include <cmath>

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
        // 2-D: axis 0 indexes independent slices
        const T* sl = s + (long long)i0 * dm.n[1] * dm.n[2];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T* row = sl + o1[b];
            acc += w1[b] * (w2[0] * row[o2[0]] + w2[1] * row[o2[1]] + w2[2] * row[o2[2]] +
                            w2[3] * row[o2[3]]);
        }
    }
    return acc;
}

// ---- tile geometry -----------------------------------------------------------
// 3-D: threads (32 x 8), each owns TZ points along z.  2-D: threads (64 x 4),
// each owns 8 points along y (tile 64 x 32).  H is the halo: the staged region
// covers departure displacements of up to H cells.
template <typename T_, int DIM_, int H>
struct Tile;
template <typename T_, int H>
struct Tile<T_, 3, H> {
    using T = T_;
    static constexpr int DIM = 3;
    static constexpr int TX = 32, TY = 8, TZ = sizeof(T) == 4 ? 8 : 4;
    static constexpr int HALO = H;
    static constexpr int RX = TX + 2 * H + 3, RY = TY + 2 * H + 3, RZ = TZ + 2 * H + 3;
    static constexpr int PTS = TZ;  // points per thread
};
template <typename T_, int H>
struct Tile<T_, 2, H> {
    using T = T_;
    static constexpr int DIM = 2;
    static constexpr int TX = 64, TY = 32, TZ = 1;
    static constexpr int HALO = H;
    static constexpr int RX = TX + 2 * H + 3, RY = TY + 2 * H + 3, RZ = 1;
    static constexpr int PTS = 8;
};

template <class C>
constexpr size_t tile_lds_bytes() {
    return sizeof(typename C::T) * C::RX * C::RY * C::RZ;
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
template <class C>
__device__ inline void stage(const Dims& dm, const typename C::T* __restrict__ src,
                             typename C::T* lds, int x0, int y0, int z0) {
    using T = typename C::T;
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
        // 2-D: axis 0 indexes independent slices (no interpolation across it)
        const int gz = C::DIM == 3 ? wrapn(z0 - C::HALO - 1 + rz, dm.n[0]) : z0;
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
template <class C>
__device__ inline typename C::T gather_lds(const typename C::T* lds, int lx, int ly, int lz,
                                           typename C::T d0, typename C::T d1, typename C::T d2) {
    using T = typename C::T;
    T wx[4], wy[4];
    const int bx = lds_axis<T, C::HALO, C::RX>(lx, d2, wx);
    const int by = lds_axis<T, C::HALO, C::RY>(ly, d1, wy);
    T acc = T(0);
    if constexpr (C::DIM == 3) {
        T wz[4];
        const int bz = lds_axis<T, C::HALO, C::RZ>(lz, d0, wz);
        const T* base = lds + (bz * C::RY + by) * C::RX + bx;
#ifdef GAN_SL_PRELOAD
        T val[64];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) val[(a * 4 + b) * 4 + c] = base[(a * C::RY + b) * C::RX + c];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            T sa = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const T* row = val + (a * 4 + b) * 4;
                sa += wy[b] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2] + wx[3] * row[3]);
            }
            acc += wz[a] * sa;
        }
#else
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
#endif
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

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b mod 8), each with its own L2.  Tiles are numbered x-fastest, then y,
// then z, and XCD k is given the contiguous range of tiles
// [k ceil(T/8), (k+1) ceil(T/8)): a slab whose halos are mostly read from
// the same L2 instead of once per XCD.
constexpr int kXcds = 8;

template <class C>
__host__ __device__ inline int tile_count(const Dims& dm) {
    const int ntx = (dm.n[2] + C::TX - 1) / C::TX;
    const int nty = (dm.n[1] + C::TY - 1) / C::TY;
    const int ntz = C::DIM == 3 ? (dm.n[0] + C::TZ - 1) / C::TZ : dm.n[0];
    return ntx * nty * ntz;
}

// Tile origin of this block and the local coordinates of the thread's k-th point.
template <class C>
struct PointMap {
    int x0, y0, z0;
    bool valid;
    __device__ PointMap(const Dims& dm) {
        const int ntx = (dm.n[2] + C::TX - 1) / C::TX;
        const int nty = (dm.n[1] + C::TY - 1) / C::TY;
        const int T = tile_count<C>(dm);
        const int per = (T + kXcds - 1) / kXcds;
        const int t = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
        valid = t < T;
        x0 = (t % ntx) * C::TX;
        y0 = ((t / ntx) % nty) * C::TY;
        z0 = (t / (ntx * nty)) * C::TZ;
    }
    __device__ void local(int k, int& lx, int& ly, int& lz) const {
        if constexpr (C::DIM == 3) {
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

template <class C>
int tile_blocks(const Dims& dm) {
    const int T = tile_count<C>(dm);
    return kXcds * ((T + kXcds - 1) / kXcds);
}

// ---- semi-Lagrangian step --------------------------------------------------------
// EPI 0: out = I[src];  1: out = fac * I[src];
// EPI 2 (source factor, src = delta): out = 1 + sgn h/2 (I[d] + d) + h^2/2 d I[d]
// `bound` >= max |disp| (cells); beyond the halo the direct gather is used.
template <class C, int EPI>
__global__ void __launch_bounds__(kThreads) sl_step_kernel(
    Dims dm, const typename C::T* __restrict__ src, const typename C::T* __restrict__ disp,
    const typename C::T* __restrict__ fac, typename C::T ht, typename C::T sgn, int bound,
    typename C::T* __restrict__ out) {
    using T = typename C::T;
    constexpr int DIM = C::DIM;
    extern __shared__ double2 sl_smem[];
    T* lds = reinterpret_cast<T*>(sl_smem);
    const PointMap<C> pm(dm);
    if (!pm.valid) return;
    const bool use_lds = bound <= C::HALO;
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
    if (use_lds) stage<C>(dm, src, lds, pm.x0, pm.y0, pm.z0);
#pragma unroll
    for (int k = 0; k < C::PTS; ++k) {
        if (!in[k]) continue;
        int lx, ly, lz;
        pm.local(k, lx, ly, lz);
        T r;
        if (use_lds) {
            r = gather_lds<C>(lds, lx, ly, lz, d0[k], d1[k], d2[k]);
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
// the predictor points only depend on u at the grid point.  ubound >= max |u|.
template <class C, bool DOX, bool DOY>
__global__ void __launch_bounds__(kThreads) characteristics_kernel(
    Dims dm, const typename C::T* __restrict__ v, typename C::T s0, typename C::T s1,
    typename C::T s2, int ubound, typename C::T* __restrict__ dX, typename C::T* __restrict__ dY) {
    using T = typename C::T;
    constexpr int DIM = C::DIM;
    extern __shared__ double2 sl_smem[];
    T* lds = reinterpret_cast<T*>(sl_smem);
    const PointMap<C> pm(dm);
    if (!pm.valid) return;
    const bool use_lds = ubound <= C::HALO;
    const long long N = dm.N;
    const T s[3] = {s0, s1, s2};
    for (int c = 0; c < DIM; ++c) {
        const T* vc = v + c * N;
        if (use_lds) {
            __syncthreads();
            stage<C>(dm, vc, lds, pm.x0, pm.y0, pm.z0);
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
                const T iv = use_lds ? gather_lds<C>(lds, lx, ly, lz, -e0, -e1, -e2)
                                     : gather_global<T, DIM>(dm, vc, i0, i1, i2, -e0, -e1, -e2);
                dX[c * N + lin] = T(-0.5) * (u[c] + s[c] * iv);
            }
            if (DOY) {
                const T iv = use_lds ? gather_lds<C>(lds, lx, ly, lz, e0, e1, e2)
                                     : gather_global<T, DIM>(dm, vc, i0, i1, i2, e0, e1, e2);
                dY[c * N + lin] = T(0.5) * (u[c] + s[c] * iv);
            }
        }
    }
}

// max_c max_i |s_c v_c(i)| (NaN/inf counted as 1e30): FP64 block partials
template <typename T>
__global__ void __launch_bounds__(kThreads) velocity_max_kernel(const T* __restrict__ v,
                                                                long long N, int dim, T s0, T s1,
                                                                T s2, double* __restrict__ partial) {
    __shared__ double sh[kThreads / 64];
    const T s[3] = {s0, s1, s2};
    double m = 0.0;
    for (int c = 0; c < dim; ++c)
        for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
             i += (long long)gridDim.x * blockDim.x) {
            double a = fabs(double(v[c * N + i]) * double(s[c]));
            if (!(a <= 1.0e30)) a = 1.0e30;
            m = fmax(m, a);
        }
    const double r = block_reduce<true>(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// Variant choice: the smallest halo that covers the bound; beyond the
// largest the widest variant runs its direct-gather path.
template <typename T, int DIM>
int pick_halo(int bound) {
    if (DIM == 2) return bound <= 4 ? 4 : 8;
    if (sizeof(T) == 8) return bound <= 1 ? 1 : 2;
    return bound <= 1 ? 1 : (bound <= 2 ? 2 : 4);
}

template <class C, bool DOX, bool DOY>
void char_launch(const Dims& dm, const typename C::T* v, const double* s, int ubound,
                 typename C::T* dX, typename C::T* dY, hipStream_t st) {
    using T = typename C::T;
    characteristics_kernel<C, DOX, DOY><<<tile_blocks<C>(dm), kThreads, tile_lds_bytes<C>(), st>>>(
        dm, v, T(s[0]), T(s[1]), T(C::DIM == 3 ? s[2] : 0.0), ubound, dX, dY);
}

template <class C>
void char_dirs(const Dims& dm, const typename C::T* v, const double* s, int ubound,
               typename C::T* dX, typename C::T* dY, hipStream_t st) {
    // 3-D: one launch per direction (each keeps one gather in flight per
    // thread); 2-D: both directions in one launch
    if (C::DIM == 3 || !(dX && dY)) {
        if (dX) char_launch<C, true, false>(dm, v, s, ubound, dX, dY, st);
        if (dY) char_launch<C, false, true>(dm, v, s, ubound, dX, dY, st);
    } else {
        char_launch<C, true, true>(dm, v, s, ubound, dX, dY, st);
    }
}

template <class C>
void step_launch(const Dims& dm, const typename C::T* src, const typename C::T* disp,
                 const typename C::T* fac, int bound, typename C::T* out, hipStream_t st) {
    using T = typename C::T;
    if (fac)
        sl_step_kernel<C, 1><<<tile_blocks<C>(dm), kThreads, tile_lds_bytes<C>(), st>>>(
            dm, src, disp, fac, T(0), T(0), bound, out);
    else
        sl_step_kernel<C, 0><<<tile_blocks<C>(dm), kThreads, tile_lds_bytes<C>(), st>>>(
            dm, src, disp, fac, T(0), T(0), bound, out);
}

template <class C>
void factor_launch(const Dims& dm, const typename C::T* delta, const typename C::T* disp,
                   double ht, double sgn, int bound, typename C::T* out, hipStream_t st) {
    using T = typename C::T;
    sl_step_kernel<C, 2><<<tile_blocks<C>(dm), kThreads, tile_lds_bytes<C>(), st>>>(
        dm, delta, disp, nullptr, T(ht), T(sgn), bound, out);
}

// Calls f(Tile<...>{}) with the variant chosen for `bound`.
template <typename T, typename F>
void dispatch_tile(const Dims& dm, int bound, F&& f) {
    if (dm.dim == 3) {
        const int h = pick_halo<T, 3>(bound);
        if (h == 1) f(Tile<T, 3, 1>{});
        else if (h == 2 || sizeof(T) == 8) f(Tile<T, 3, 2>{});
        else f(Tile<T, 3, 4>{});
    } else {
        if (pick_halo<T, 2>(bound) == 4) f(Tile<T, 2, 4>{});
        else f(Tile<T, 2, 8>{});
    }
}

}  // namespace

int displacement_bound(double umax, int dim) {
    // |X| = |u(i) + I[u](xi*)| / 2 <= (1 + 1.25^d) max|u| / 2: the cubic
    // Lagrange weights have absolute sum at most 1.25 per axis
    if (!(umax <= 1.0e6)) return 1 << 20;
    const double f = 0.5 * (1.0 + std::pow(1.25, dim));
    return static_cast<int>(std::ceil(f * umax * (1.0 + 1e-6)));
}

template <typename T>
hipError_t launch_velocity_max(const Dims& dm, const T* v, const double* s, double* partial,
                               double* res, hipStream_t st) {
    const int nb = reduction_blocks(dm.N);
    velocity_max_kernel<T><<<nb, kThreads, 0, st>>>(v, dm.N, dm.dim, T(s[0]), T(s[1]),
                                                    T(dm.dim == 3 ? s[2] : 0.0), partial);
    finish_kernel<true><<<1, 1024, 0, st>>>(partial, nb, 1, res);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_characteristics(const Dims& dm, const T* v, const double* s, int ubound, T* dX,
                                  T* dY, hipStream_t st) {
    dispatch_tile<T>(dm, ubound, [&](auto tile) {
        char_dirs<decltype(tile)>(dm, v, s, ubound, dX, dY, st);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sl_step(const Dims& dm, const T* src, const T* disp, const T* fac, int bound,
                          T* out, hipStream_t st) {
    dispatch_tile<T>(dm, bound, [&](auto tile) {
        step_launch<decltype(tile)>(dm, src, disp, fac, bound, out, st);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_source_factor(const Dims& dm, const T* delta, const T* disp, double ht,
                                double sgn, int bound, T* out, hipStream_t st) {
    dispatch_tile<T>(dm, bound, [&](auto tile) {
        factor_launch<decltype(tile)>(dm, delta, disp, ht, sgn, bound, out, st);
    });
    return hipGetLastError();
}

#define GAN_INST(T)                                                                               \
    template hipError_t launch_velocity_max<T>(const Dims&, const T*, const double*, double*,     \
                                               double*, hipStream_t);                             \
    template hipError_t launch_characteristics<T>(const Dims&, const T*, const double*, int, T*,  \
                                                  T*, hipStream_t);                               \
    template hipError_t launch_sl_step<T>(const Dims&, const T*, const T*, const T*, int, T*,     \
                                          hipStream_t);                                           \
    template hipError_t launch_source_factor<T>(const Dims&, const T*, const T*, double, double,  \
                                                int, T*, hipStream_t);
GAN_INST(float)
GAN_INST(double)
#undef GAN_INST

}  // namespace gan
