// Shared device/host definitions of the GA-NGMRES transport library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gan {

// Internal grids are always three-dimensional with extents n[0..2] and the
// last axis contiguous.  A 2-D problem of shape (n1, n2) is stored as
// (1, n1, n2); vector component c of a d-dimensional field acts along the
// internal axis 3 - d + c.
struct Dims {
    int n[3];
    int dim;
    long long N;       // n0 n1 n2
    int n2h;           // n2/2 + 1 (half-spectrum length of the last axis)
    long long NH;      // n0 n1 n2h
    int tile;          // 2-D gather tiles: points per thread (8, 4 or 2; 0: 8)
};

// 2-D gather tile height in points per thread when no variant was chosen.
constexpr int kTile2Default = 8;

inline __host__ __device__ int comp_axis(int dim, int c) { return 3 - dim + c; }

template <typename T>
struct C2 {
    T x, y;
};

template <typename T>
__host__ __device__ inline C2<T> cmk(T a, T b) {
    C2<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__host__ __device__ inline C2<T> cadd(C2<T> a, C2<T> b) { return cmk(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ inline C2<T> csub(C2<T> a, C2<T> b) { return cmk(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ inline C2<T> cmul(C2<T> a, C2<T> b) {
    return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ inline C2<T> cscale(C2<T> a, T s) { return cmk(a.x * s, a.y * s); }
template <typename T>
__host__ __device__ inline C2<T> cconj(C2<T> a) { return cmk(a.x, -a.y); }
// multiply by i*s
template <typename T>
__host__ __device__ inline C2<T> cmuli(C2<T> a, T s) { return cmk(-a.y * s, a.x * s); }

// Signed wavenumber of index i on an axis of length n (Nyquist is +n/2).
__host__ __device__ inline int wavenumber(int i, int n) { return (2 * i <= n) ? i : i - n; }
// Wavenumber for odd derivatives: Nyquist set to zero.
__host__ __device__ inline int wavenumber_odd(int i, int n) {
    return (2 * i == n) ? 0 : ((2 * i < n) ? i : i - n);
}

// Non-negative remainder, valid for every int a (n > 0).
__host__ __device__ inline int pmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

constexpr int kMaxRadices = 16;

// Mixed-radix plan of a length-L transform: radices applied in order, and a
// table tw[m] = exp(-2 pi i m / L) computed in FP64 on the host.
template <typename T>
struct FftPlan {
    int L;
    int nrad;
    int rad[kMaxRadices];
    const C2<T>* tw;
};

}  // namespace gan
