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
// Launch shape: one thread per output point, blocks of 64 x 4 along the two
// fastest axes (a wavefront covers 64 contiguous points of one row), grid.z
// runs over the slowest axis.  Source reads go through L1/L2: a departure
// stencil overlaps its neighbours' when the displacement is smooth.
#include "launch.hpp"

namespace gan {

namespace {

template <typename T>
__device__ inline void lagrange4(T t, T* w) {
    const T tp1 = t + T(1), tm1 = t - T(1), tm2 = t - T(2);
    const T sixth = T(1.0 / 6.0);
    w[0] = -t * tm1 * tm2 * sixth;
    w[1] = tp1 * tm1 * tm2 * T(0.5);
    w[2] = -tp1 * t * tm2 * T(0.5);
    w[3] = tp1 * t * tm1 * sixth;
}

// Taps along one axis: element offsets (already times the axis stride) and
// weights for a departure displacement `disp` from grid index i.
template <typename T>
__device__ inline void axis_taps(int i, T disp, int n, int stride, int* off, T* w) {
    disp = fmin(fmax(disp, T(-1.0e7)), T(1.0e7));
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

struct Idx {
    int i0, i1, i2;
    int lin;
};

__device__ inline bool thread_point(const Dims& dm, Idx& p) {
    p.i2 = blockIdx.x * blockDim.x + threadIdx.x;
    p.i1 = blockIdx.y * blockDim.y + threadIdx.y;
    p.i0 = blockIdx.z;
    if (p.i2 >= dm.n[2] || p.i1 >= dm.n[1]) return false;
    p.lin = (p.i0 * dm.n[1] + p.i1) * dm.n[2] + p.i2;
    return true;
}

// Interpolate NF fields (stride fstride apart) at grid point p displaced by
// (d0, d1, d2) cells along the internal axes (d0 unused for DIM == 2).
template <typename T, int DIM, int NF>
__device__ inline void gather(const Dims& dm, const T* src, long long fstride, const Idx& p, T d0,
                              T d1, T d2, T* out) {
    int o1[4], o2[4];
    T w1[4], w2[4];
    axis_taps(p.i1, d1, dm.n[1], dm.n[2], o1, w1);
    axis_taps(p.i2, d2, dm.n[2], 1, o2, w2);
    if constexpr (DIM == 3) {
        int o0[4];
        T w0[4];
        axis_taps(p.i0, d0, dm.n[0], dm.n[1] * dm.n[2], o0, w0);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T* s = src + f * fstride;
            T acc = T(0);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                T sa = T(0);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const T* row = s + o0[a] + o1[b];
                    T sb = w2[0] * row[o2[0]] + w2[1] * row[o2[1]] + w2[2] * row[o2[2]] +
                           w2[3] * row[o2[3]];
                    sa += w1[b] * sb;
                }
                acc += w0[a] * sa;
            }
            out[f] = acc;
        }
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T* s = src + f * fstride;
            T acc = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const T* row = s + o1[b];
                T sb = w2[0] * row[o2[0]] + w2[1] * row[o2[1]] + w2[2] * row[o2[2]] +
                       w2[3] * row[o2[3]];
                acc += w1[b] * sb;
            }
            out[f] = acc;
        }
    }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) characteristics_kernel(Dims dm, const T* __restrict__ v,
                                                              T s0, T s1, T s2, T* __restrict__ dX,
                                                              T* __restrict__ dY) {
    Idx p;
    if (!thread_point(dm, p)) return;
    const long long N = dm.N;
    const T s[3] = {s0, s1, s2};
    T u[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) u[c] = v[c * N + p.lin] * s[c];
    // displacement along internal axes: components map to the last DIM axes
    T iv[DIM];
    if constexpr (DIM == 3) {
        gather<T, 3, 3>(dm, v, N, p, -u[0], -u[1], -u[2], iv);
    } else {
        gather<T, 2, 2>(dm, v, N, p, T(0), -u[0], -u[1], iv);
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) dX[c * N + p.lin] = T(-0.5) * (u[c] + s[c] * iv[c]);
    if (dY) {
        if constexpr (DIM == 3) {
            gather<T, 3, 3>(dm, v, N, p, u[0], u[1], u[2], iv);
        } else {
            gather<T, 2, 2>(dm, v, N, p, T(0), u[0], u[1], iv);
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) dY[c * N + p.lin] = T(0.5) * (u[c] + s[c] * iv[c]);
    }
}

template <typename T, int DIM, bool FAC>
__global__ void __launch_bounds__(256) sl_step_kernel(Dims dm, const T* __restrict__ src,
                                                      const T* __restrict__ disp,
                                                      const T* __restrict__ fac, T* __restrict__ out) {
    Idx p;
    if (!thread_point(dm, p)) return;
    const long long N = dm.N;
    T r;
    if constexpr (DIM == 3) {
        gather<T, 3, 1>(dm, src, 0, p, disp[p.lin], disp[N + p.lin], disp[2 * N + p.lin], &r);
    } else {
        gather<T, 2, 1>(dm, src, 0, p, T(0), disp[p.lin], disp[N + p.lin], &r);
    }
    if constexpr (FAC) r *= fac[p.lin];
    out[p.lin] = r;
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) factor_kernel(Dims dm, const T* __restrict__ delta,
                                                     const T* __restrict__ disp, T ht, T sgn,
                                                     T* __restrict__ out) {
    Idx p;
    if (!thread_point(dm, p)) return;
    const long long N = dm.N;
    T dd;
    if constexpr (DIM == 3) {
        gather<T, 3, 1>(dm, delta, 0, p, disp[p.lin], disp[N + p.lin], disp[2 * N + p.lin], &dd);
    } else {
        gather<T, 2, 1>(dm, delta, 0, p, T(0), disp[p.lin], disp[N + p.lin], &dd);
    }
    const T d = delta[p.lin];
    out[p.lin] = T(1) + sgn * T(0.5) * ht * (dd + d) + T(0.5) * ht * ht * d * dd;
}

inline void point_grid(const Dims& dm, dim3& g, dim3& b) {
    b = dim3(64, 4, 1);
    g = dim3((dm.n[2] + 63) / 64, (dm.n[1] + 3) / 4, dm.n[0]);
}

}  // namespace

template <typename T>
hipError_t launch_characteristics(const Dims& dm, const T* v, const double* s, T* dX, T* dY,
                                  hipStream_t st) {
    dim3 g, b;
    point_grid(dm, g, b);
    if (dm.dim == 3)
        characteristics_kernel<T, 3><<<g, b, 0, st>>>(dm, v, T(s[0]), T(s[1]), T(s[2]), dX, dY);
    else
        characteristics_kernel<T, 2><<<g, b, 0, st>>>(dm, v, T(s[0]), T(s[1]), T(0), dX, dY);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sl_step(const Dims& dm, const T* src, const T* disp, const T* fac, T* out,
                          hipStream_t st) {
    dim3 g, b;
    point_grid(dm, g, b);
    if (dm.dim == 3) {
        if (fac) sl_step_kernel<T, 3, true><<<g, b, 0, st>>>(dm, src, disp, fac, out);
        else sl_step_kernel<T, 3, false><<<g, b, 0, st>>>(dm, src, disp, fac, out);
    } else {
        if (fac) sl_step_kernel<T, 2, true><<<g, b, 0, st>>>(dm, src, disp, fac, out);
        else sl_step_kernel<T, 2, false><<<g, b, 0, st>>>(dm, src, disp, fac, out);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_source_factor(const Dims& dm, const T* delta, const T* disp, double ht,
                                double sgn, T* out, hipStream_t st) {
    dim3 g, b;
    point_grid(dm, g, b);
    if (dm.dim == 3) factor_kernel<T, 3><<<g, b, 0, st>>>(dm, delta, disp, T(ht), T(sgn), out);
    else factor_kernel<T, 2><<<g, b, 0, st>>>(dm, delta, disp, T(ht), T(sgn), out);
    return hipGetLastError();
}

#define GAN_INST(T)                                                                             \
    template hipError_t launch_characteristics<T>(const Dims&, const T*, const double*, T*, T*, \
                                                  hipStream_t);                                 \
    template hipError_t launch_sl_step<T>(const Dims&, const T*, const T*, const T*, T*,        \
                                          hipStream_t);                                         \
    template hipError_t launch_source_factor<T>(const Dims&, const T*, const T*, double, double, \
                                                T*, hipStream_t);
GAN_INST(float)
GAN_INST(double)
#undef GAN_INST

}  // namespace gan
