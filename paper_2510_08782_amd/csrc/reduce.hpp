// Deterministic FP64 block reductions (wavefront shuffles, fixed tree).
#pragma once

#include "common.hpp"
#include "group.hpp"

namespace gan {

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    return x;
}
__device__ inline double wave_max(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_down(x, o, 64));
    return x;
}

// Block-wide sum (or max) of one value per thread; the result is valid in
// thread 0.  sh must hold blockDim.x / 64 doubles.  Every thread must call it.
template <bool MAX>
__device__ inline double block_reduce(double x, double* sh) {
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    x = MAX ? wave_max(x) : wave_sum(x);
    if (lane == 0) sh[wid] = x;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        r = sh[0];
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 1; i < nw; ++i) r = MAX ? fmax(r, sh[i]) : r + sh[i];
    }
    __syncthreads();
    return r;
}

// Stage 2: res[q] = fold of partial[q*nb .. q*nb + nb) for q < nq; workgroup
// b of 1024 threads folds q = b, b + gx, ... (launch finish_blocks(nq) of
// them, so that the quantities fold in parallel).
struct FinishArgs {
    const double* partial;
    int nb, nq;
    double* res;
};
template <bool MAX>
struct FinishBody {
    static constexpr int kBlock = 1024;
    using Args = FinishArgs;
    __device__ __forceinline__ static void run(const Args& a, const Blk& bk) {
        __shared__ double sh[1024 / 64];
        for (int q = bk.x; q < a.nq; q += bk.gx) {
            double x = MAX ? -INFINITY : 0.0;
            for (int i = threadIdx.x; i < a.nb; i += blockDim.x)
                x = MAX ? fmax(x, a.partial[(long long)q * a.nb + i])
                        : x + a.partial[(long long)q * a.nb + i];
            const double r = block_reduce<MAX>(x, sh);
            if (threadIdx.x == 0) a.res[q] = r;
        }
    }
};

inline unsigned finish_blocks(long long nq) {
    return (unsigned)(nq < 1 ? 1 : (nq > 4096 ? 4096 : nq));
}

// Fold nq quantities of nb partials each into res.
template <bool MAX>
inline void launch_finish(const double* partial, int nb, int nq, double* res, hipStream_t st) {
    submit<FinishBody<MAX>>(dim3(finish_blocks(nq)), 0, st, FinishArgs{partial, nb, nq, res});
}

}  // namespace gan
