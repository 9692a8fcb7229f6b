// FP64-accumulated reductions and vector updates.
//
// Reductions are deterministic: stage 1 runs a fixed number of blocks
// (a function of n only) with a grid-stride loop and a fixed
// wavefront-shuffle tree, writing one partial per block; stage 2 is a single
// block that folds the partials in a fixed order.  Repeated calls on the same
// data are therefore bitwise identical.
#include "launch.hpp"
#include "reduce.hpp"

namespace gan {

namespace {

constexpr int kRedThreads = 256;
constexpr int kMaxRedBlocks = 1024;

template <typename T>
__global__ void __launch_bounds__(kRedThreads) sumsq_diff_kernel(const T* __restrict__ a,
                                                                 const T* __restrict__ b,
                                                                 T* __restrict__ lam, long long n,
                                                                 double* __restrict__ partial) {
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const T d = b[i] - a[i];
        if (lam) lam[i] = d;
        const double dd = static_cast<double>(d);
        acc += dd * dd;
    }
    const double r = block_reduce<false>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads) dot_kernel(const T* __restrict__ a,
                                                          const T* __restrict__ b, long long n,
                                                          double* __restrict__ partial) {
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        acc += static_cast<double>(a[i]) * static_cast<double>(b[i]);
    const double r = block_reduce<false>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads) maxabs_kernel(const T* __restrict__ a, long long n,
                                                             double* __restrict__ partial) {
    __shared__ double sh[kRedThreads / 64];
    double m = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double x = fabs(static_cast<double>(a[i]));
        if (!(x <= 1.0e308)) x = INFINITY;  // NaN and inf both count as inf
        m = fmax(m, x);
    }
    const double r = block_reduce<true>(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

template <typename T, int K>
struct VecList {
    const T* p[K];
};

template <typename T, int K>
__global__ void __launch_bounds__(kRedThreads) gram_kernel(VecList<T, K> vl, long long n,
                                                           double* __restrict__ partial) {
    __shared__ double sh[kRedThreads / 64];
    constexpr int NP = K * (K + 1) / 2;
    double acc[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[q] = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double x[K];
#pragma unroll
        for (int a = 0; a < K; ++a) x[a] = static_cast<double>(vl.p[a][i]);
        int q = 0;
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int b = a; b < K; ++b) acc[q++] += x[a] * x[b];
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const double r = block_reduce<false>(acc[q], sh);
        if (threadIdx.x == 0) partial[(long long)q * gridDim.x + blockIdx.x] = r;
    }
}

template <typename T>
__global__ void axpy_kernel(const T* __restrict__ a, T s, const T* __restrict__ b,
                            T* __restrict__ out, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = a[i] + s * b[i];
}

constexpr int kMaxCombine = 65;
template <typename T>
struct CombineArgs {
    const T* x[kMaxCombine];
    T c[kMaxCombine];
};

template <typename T>
__global__ void combine_kernel(const T* __restrict__ q, CombineArgs<T> ca, int K,
                               T* __restrict__ out, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const T qi = q[i];
        T acc = qi;
        for (int k = 0; k < K; ++k) acc += ca.c[k] * (qi - ca.x[k][i]);
        out[i] = acc;
    }
}

inline int stream_blocks(long long n) {
    long long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return static_cast<int>(b);
}

template <typename T, int K>
hipError_t gram_k(const T* const* vecs, long long n, double* partial, double* res,
                  hipStream_t st) {
    VecList<T, K> vl;
    for (int a = 0; a < K; ++a) vl.p[a] = vecs[a];
    const int nb = reduction_blocks(n);
    gram_kernel<T, K><<<nb, kRedThreads, 0, st>>>(vl, n, partial);
    finish_kernel<false><<<1, 1024, 0, st>>>(partial, nb, K * (K + 1) / 2, res);
    return hipGetLastError();
}

}  // namespace

int reduction_blocks(long long n) {
    long long b = (n + kRedThreads * 8 - 1) / (kRedThreads * 8);
    if (b > kMaxRedBlocks) b = kMaxRedBlocks;
    if (b < 1) b = 1;
    return static_cast<int>(b);
}

template <typename T>
hipError_t launch_sumsq_diff(const T* a, const T* b, T* lam, long long n, double* partial,
                             double* res, hipStream_t st) {
    const int nb = reduction_blocks(n);
    sumsq_diff_kernel<T><<<nb, kRedThreads, 0, st>>>(a, b, lam, n, partial);
    finish_kernel<false><<<1, 1024, 0, st>>>(partial, nb, 1, res);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dot(const T* a, const T* b, long long n, double* partial, double* res,
                      hipStream_t st) {
    const int nb = reduction_blocks(n);
    dot_kernel<T><<<nb, kRedThreads, 0, st>>>(a, b, n, partial);
    finish_kernel<false><<<1, 1024, 0, st>>>(partial, nb, 1, res);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_maxabs(const T* a, long long n, double* partial, double* res, hipStream_t st) {
    const int nb = reduction_blocks(n);
    maxabs_kernel<T><<<nb, kRedThreads, 0, st>>>(a, n, partial);
    finish_kernel<true><<<1, 1024, 0, st>>>(partial, nb, 1, res);
    return hipGetLastError();
}

// The packed Gram kernel writes the upper triangle in row order; the host
// unpacks.  Here res receives K(K+1)/2 packed values.
template <typename T>
hipError_t launch_gram(const T* const* vecs, int K, long long n, double* partial, double* res,
                       hipStream_t st) {
    switch (K) {
        case 1: return gram_k<T, 1>(vecs, n, partial, res, st);
        case 2: return gram_k<T, 2>(vecs, n, partial, res, st);
        case 3: return gram_k<T, 3>(vecs, n, partial, res, st);
        case 4: return gram_k<T, 4>(vecs, n, partial, res, st);
        case 5: return gram_k<T, 5>(vecs, n, partial, res, st);
        case 6: return gram_k<T, 6>(vecs, n, partial, res, st);
        case 7: return gram_k<T, 7>(vecs, n, partial, res, st);
        case 8: return gram_k<T, 8>(vecs, n, partial, res, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_axpy(const T* a, double s, const T* b, T* out, long long n, hipStream_t st) {
    axpy_kernel<T><<<stream_blocks(n), 256, 0, st>>>(a, T(s), b, out, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_combine(const T* q, const T* const* x, const double* c, int K, T* out,
                          long long n, hipStream_t st) {
    if (K < 0 || K > kMaxCombine) return hipErrorInvalidValue;
    CombineArgs<T> ca;
    for (int k = 0; k < kMaxCombine; ++k) {
        ca.x[k] = k < K ? x[k] : nullptr;
        ca.c[k] = k < K ? T(c[k]) : T(0);
    }
    combine_kernel<T><<<stream_blocks(n), 256, 0, st>>>(q, ca, K, out, n);
    return hipGetLastError();
}

#define GAN_INST(T)                                                                             \
    template hipError_t launch_sumsq_diff<T>(const T*, const T*, T*, long long, double*, double*, \
                                             hipStream_t);                                      \
    template hipError_t launch_dot<T>(const T*, const T*, long long, double*, double*,          \
                                      hipStream_t);                                             \
    template hipError_t launch_maxabs<T>(const T*, long long, double*, double*, hipStream_t);   \
    template hipError_t launch_gram<T>(const T* const*, int, long long, double*, double*,       \
                                       hipStream_t);                                            \
    template hipError_t launch_axpy<T>(const T*, double, const T*, T*, long long, hipStream_t);  \
    template hipError_t launch_combine<T>(const T*, const T* const*, const double*, int, T*,    \
                                          long long, hipStream_t);
GAN_INST(float)
GAN_INST(double)
#undef GAN_INST

}  // namespace gan
