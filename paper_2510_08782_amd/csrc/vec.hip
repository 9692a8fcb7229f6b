// FP64-accumulated reductions and vector updates.
//
// Reductions are deterministic: stage 1 runs a fixed number of blocks per
// segment (a function of the sizes only) with a grid-stride loop and a fixed
// wavefront-shuffle tree, writing one partial per block; stage 2 is a single
// block that folds the partials in a fixed order.  Repeated calls on the same
// data are therefore bitwise identical.  Segments are the independent
// problems of a batch (one segment for a single problem).
#include <algorithm>

#include "launch.hpp"
#include "group.hpp"
#include "reduce.hpp"

namespace gan {

namespace {

constexpr int kRedThreads = 256;
constexpr int kMaxRedBlocks = 1024;
constexpr long long kPartialCap = 64 * 1024;  // doubles in the partials buffer

// Element (c, s, i) of a segmented array (see Seg).
__device__ inline long long seg_at(const Seg& g, int c, int s, long long i) {
    return c * g.cstride + s * g.seglen + i;
}

// Every reduction kernel runs gridDim.y = nseg rows of gridDim.x blocks; block
// 16 bytes of T, moved with one load or store (elements W = 16 / sizeof(T))
template <typename T>
struct alignas(16) Vec16 {
    static constexpr int W = 16 / (int)sizeof(T);
    T v[W];
};
// rows of a segmented array can move as Vec16 when every row start is
// 16-byte aligned
template <typename T>
bool vec16_rows(const Seg& g, std::initializer_list<const void*> ptrs) {
    constexpr int W = 16 / (int)sizeof(T);
    if (g.seglen % W != 0 || g.cstride % W != 0) return false;
    for (const void* p : ptrs)
        if (reinterpret_cast<unsigned long long>(p) & 15) return false;
    return true;
}

// (x, s) strides over segment s and writes partial[(q nseg + s) gridDim.x + x]
// for its quantity q.
// f(e, w) on every element of segment s, element e of the array, w its
// position in a 16-byte group; with vec the rows move as Vec16 (vec16_rows).
// f gets the element's index and returns nothing; the loads are in f.
template <typename T, typename F>
__device__ inline void seg_for(const Blk& bk, const Seg& g, int s, bool vec, F&& f) {
    if (vec) {
        constexpr int W = Vec16<T>::W;
        const long long nv = g.seglen / W;
        for (int c = 0; c < g.ncomp; ++c)
            for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < nv;
                 i += (long long)bk.gx * blockDim.x)
                f(seg_at(g, c, s, 0) / W + i, true);
    } else {
        for (int c = 0; c < g.ncomp; ++c)
            for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < g.seglen;
                 i += (long long)bk.gx * blockDim.x)
                f(seg_at(g, c, s, i), false);
    }
}

template <typename T>
struct SumsqDiffArgs {
    const T* a;
    const T* b;
    T* lam;
    Seg g;
    int vec;
    double* partial;
};
template <typename T>
struct SumsqDiffBody {
    static constexpr int kBlock = kRedThreads;
    using Args = SumsqDiffArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const T* __restrict__ a = args_.a;
        const T* __restrict__ b = args_.b;
        T* __restrict__ lam = args_.lam;
        const Seg& g = args_.g;
        int vec = args_.vec;
        double* __restrict__ partial = args_.partial;
        __shared__ double sh[kRedThreads / 64];
        const int s = bk.y;
        double acc = 0.0;
        seg_for<T>(bk, g, s, vec != 0, [&](long long e, bool v) {
            if (v) {
                const Vec16<T> av = reinterpret_cast<const Vec16<T>*>(a)[e];
                const Vec16<T> bv = reinterpret_cast<const Vec16<T>*>(b)[e];
                Vec16<T> dv;
    #pragma unroll
                for (int w = 0; w < Vec16<T>::W; ++w) {
                    dv.v[w] = bv.v[w] - av.v[w];
                    const double dd = static_cast<double>(dv.v[w]);
                    acc += dd * dd;
                }
                if (lam) reinterpret_cast<Vec16<T>*>(lam)[e] = dv;
            } else {
                const T d = b[e] - a[e];
                if (lam) lam[e] = d;
                const double dd = static_cast<double>(d);
                acc += dd * dd;
            }
        });
        const double r = block_reduce<false>(acc, sh);
        if (threadIdx.x == 0) partial[(long long)s * bk.gx + bk.x] = r;
    }
};

template <typename T>
struct DotArgs {
    const T* a;
    const T* b;
    Seg g;
    int vec;
    double* partial;
};
template <typename T>
struct DotBody {
    static constexpr int kBlock = kRedThreads;
    using Args = DotArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const T* __restrict__ a = args_.a;
        const T* __restrict__ b = args_.b;
        const Seg& g = args_.g;
        int vec = args_.vec;
        double* __restrict__ partial = args_.partial;
        __shared__ double sh[kRedThreads / 64];
        const int s = bk.y;
        double acc = 0.0;
        seg_for<T>(bk, g, s, vec != 0, [&](long long e, bool v) {
            if (v) {
                const Vec16<T> av = reinterpret_cast<const Vec16<T>*>(a)[e];
                const Vec16<T> bv = reinterpret_cast<const Vec16<T>*>(b)[e];
    #pragma unroll
                for (int w = 0; w < Vec16<T>::W; ++w)
                    acc += static_cast<double>(av.v[w]) * static_cast<double>(bv.v[w]);
            } else {
                acc += static_cast<double>(a[e]) * static_cast<double>(b[e]);
            }
        });
        const double r = block_reduce<false>(acc, sh);
        if (threadIdx.x == 0) partial[(long long)s * bk.gx + bk.x] = r;
    }
};

template <typename T>
struct MaxabsArgs {
    const T* a;
    Seg g;
    int vec;
    double* partial;
};
template <typename T>
struct MaxabsBody {
    static constexpr int kBlock = kRedThreads;
    using Args = MaxabsArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const T* __restrict__ a = args_.a;
        const Seg& g = args_.g;
        int vec = args_.vec;
        double* __restrict__ partial = args_.partial;
        __shared__ double sh[kRedThreads / 64];
        const int s = bk.y;
        T m = T(0);
        bool bad = false;
        seg_for<T>(bk, g, s, vec != 0, [&](long long e, bool v) {
            if (v) {
                const Vec16<T> av = reinterpret_cast<const Vec16<T>*>(a)[e];
    #pragma unroll
                for (int w = 0; w < Vec16<T>::W; ++w) {
                    const T x = fabs(av.v[w]);
                    bad = bad || !(x == x);
                    m = fmax(m, x);
                }
            } else {
                const T x = fabs(a[e]);
                bad = bad || !(x == x);
                m = fmax(m, x);
            }
        });
        // NaN and inf both count as inf
        const double r = block_reduce<true>(bad ? INFINITY : static_cast<double>(m), sh);
        if (threadIdx.x == 0) partial[(long long)s * bk.gx + bk.x] = r;
    }
};

template <typename T, int K>
struct VecList {
    const T* p[K];
};

// Gram matrix of K > 8 vectors (up to the largest window plus two) in one
// pass over the data.  A block stages a chunk of kGramE elements of every
// vector in LDS (as FP64), then its threads form the chunk's products in 4 x 4
// tiles of vector pairs: the upper triangle of the padded K x K matrix has
// ntiles tiles, each owned by S = blockDim / ntiles threads that split the
// chunk's elements.  After the last chunk the S partial tiles are folded in
// a fixed order, so the result does not depend on timing.
constexpr int kGramE = 128;
constexpr long long kGramPartialCap = kGramPartialDoubles;
template <typename T>
struct PtrList {
    const T* p[kMaxGram];
};

__host__ __device__ inline int packed_pair(int a, int b, int K) { return a * K - a * (a - 1) / 2 + (b - a); }

template <typename T>
struct GramBigArgs {
    PtrList<T> pl;
    int K;
    Seg g;
    double* partial;
};
template <typename T>
struct GramBigBody {
    static constexpr int kBlock = kRedThreads;
    using Args = GramBigArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const PtrList<T>& pl = args_.pl;
        int K = args_.K;
        const Seg& g = args_.g;
        double* __restrict__ partial = args_.partial;
        extern __shared__ double gsm[];  // max(Kp kGramE, kRedThreads 16) doubles
        const int s = bk.y;
        const int nt = (K + 3) / 4, Kp = 4 * nt;
        const int ntiles = nt * (nt + 1) / 2;
        const int S = kRedThreads / ntiles;
        const int t = threadIdx.x;
        const bool active = t < ntiles * S;
        const int tile = active ? t / S : 0, slice = active ? t % S : 0;
        int ta = 0, rem = tile;
        while (rem >= nt - ta) {
            rem -= nt - ta;
            ++ta;
        }
        const int tb = ta + rem;
        double acc[4][4];
    #pragma unroll
        for (int r = 0; r < 4; ++r)
    #pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
        for (int i = t; i < (Kp - K) * kGramE; i += blockDim.x) gsm[K * kGramE + i] = 0.0;
        const long long nch = (g.seglen + kGramE - 1) / kGramE;
        const long long total = nch * g.ncomp;
        for (long long ch = bk.x; ch < total; ch += bk.gx) {
            const int c = static_cast<int>(ch / nch);
            const long long i0 = (ch % nch) * kGramE;
            const long long base = seg_at(g, c, s, i0);
            const int len = static_cast<int>(min(static_cast<long long>(kGramE), g.seglen - i0));
            __syncthreads();  // the previous chunk has been read
            for (int idx = t; idx < K * kGramE; idx += blockDim.x) {
                const int a = idx / kGramE, e = idx % kGramE;
                gsm[idx] = e < len ? static_cast<double>(pl.p[a][base + e]) : 0.0;
            }
            __syncthreads();
            if (active) {
                const double* xa = gsm + 4 * ta * kGramE;
                const double* xb = gsm + 4 * tb * kGramE;
                for (int e = slice; e < len; e += S) {
                    double x[4], y[4];
    #pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        x[r] = xa[r * kGramE + e];
                        y[r] = xb[r * kGramE + e];
                    }
    #pragma unroll
                    for (int r = 0; r < 4; ++r)
    #pragma unroll
                        for (int c2 = 0; c2 < 4; ++c2) acc[r][c2] = fma(x[r], y[c2], acc[r][c2]);
                }
            }
        }
        __syncthreads();
        if (active) {
    #pragma unroll
            for (int q = 0; q < 16; ++q) gsm[t * 16 + q] = acc[q / 4][q % 4];
        }
        __syncthreads();
        if (active && slice == 0) {
            for (int q = 0; q < 16; ++q) {
                double sum = gsm[(tile * S) * 16 + q];
                for (int j = 1; j < S; ++j) sum += gsm[(tile * S + j) * 16 + q];
                const int a = 4 * ta + q / 4, b = 4 * tb + q % 4;
                if (a < K && b < K && a <= b)
                    partial[((long long)packed_pair(a, b, K) * bk.gy + s) * bk.gx + bk.x] = sum;
            }
        }
    }
};

template <typename T, int K>
struct GramArgs {
    VecList<T, K> vl;
    Seg g;
    int vec;
    double* partial;
};
template <typename T, int K>
struct GramBody {
    static constexpr int kBlock = kRedThreads;
    using Args = GramArgs<T, K>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const VecList<T, K>& vl = args_.vl;
        const Seg& g = args_.g;
        int vec = args_.vec;
        double* __restrict__ partial = args_.partial;
        __shared__ double sh[kRedThreads / 64];
        constexpr int NP = K * (K + 1) / 2;
        const int s = bk.y;
        double acc[NP];
    #pragma unroll
        for (int q = 0; q < NP; ++q) acc[q] = 0.0;
        auto add = [&](const double (&x)[K]) {
            int q = 0;
    #pragma unroll
            for (int a = 0; a < K; ++a)
    #pragma unroll
                for (int b = a; b < K; ++b) acc[q++] += x[a] * x[b];
        };
        if (vec) {
            constexpr int W = Vec16<T>::W;
            const long long nv = g.seglen / W;
            for (int c = 0; c < g.ncomp; ++c)
                for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < nv;
                     i += (long long)bk.gx * blockDim.x) {
                    const long long e = seg_at(g, c, s, 0) / W + i;
                    Vec16<T> xv[K];
    #pragma unroll
                    for (int a = 0; a < K; ++a) xv[a] = reinterpret_cast<const Vec16<T>*>(vl.p[a])[e];
    #pragma unroll
                    for (int w = 0; w < W; ++w) {
                        double x[K];
    #pragma unroll
                        for (int a = 0; a < K; ++a) x[a] = static_cast<double>(xv[a].v[w]);
                        add(x);
                    }
                }
        } else {
            for (int c = 0; c < g.ncomp; ++c)
                for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < g.seglen;
                     i += (long long)bk.gx * blockDim.x) {
                    const long long e = seg_at(g, c, s, i);
                    double x[K];
    #pragma unroll
                    for (int a = 0; a < K; ++a) x[a] = static_cast<double>(vl.p[a][e]);
                    add(x);
                }
        }
    #pragma unroll
        for (int q = 0; q < NP; ++q) {
            const double r = block_reduce<false>(acc[q], sh);
            if (threadIdx.x == 0)
                partial[((long long)q * bk.gy + s) * bk.gx + bk.x] = r;
        }
    }
};

// Segment-wise vector updates: gridDim.y = ncomp * nseg rows, row y covers
// component y / nseg of segment y % nseg.
template <typename T>
struct AxpyArgs {
    const T* a;
    SegCoef sc;
    const T* b;
    T* out;
    Seg g;
};
template <typename T>
struct AxpyBody {
    static constexpr int kBlock = 256;
    using Args = AxpyArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const T* __restrict__ a = args_.a;
        const SegCoef& sc = args_.sc;
        const T* __restrict__ b = args_.b;
        T* __restrict__ out = args_.out;
        const Seg& g = args_.g;
        const int c = bk.y / g.nseg, s = bk.y % g.nseg;
        const T k = T(sc.c[s]);
        const long long base = c * g.cstride + s * g.seglen;
        for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < g.seglen;
             i += (long long)bk.gx * blockDim.x)
            out[base + i] = a[base + i] + k * b[base + i];
    }
};

template <typename T>
struct OuterArgs {
    const T* g;
    const T* x;
    T* out;
    int d;
    long long n;
};
template <typename T>
struct OuterBody {
    static constexpr int kBlock = 256;
    using Args = OuterArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const T* __restrict__ g = args_.g;
        const T* __restrict__ x = args_.x;
        T* __restrict__ out = args_.out;
        int d = args_.d;
        long long n = args_.n;
        for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < n;
             i += (long long)bk.gx * blockDim.x) {
            T dot = T(0);
            for (int j = 0; j < d; ++j) dot += g[j * n + i] * x[j * n + i];
            for (int c = 0; c < d; ++c) out[c * n + i] = g[c * n + i] * dot;
        }
    }
};

constexpr int kMaxCombine = 65;
template <typename T>
struct CombinePtrs {
    const T* x[kMaxCombine];
};

// out = q + sum_k coef[k nseg + s] (q - x_k) on segment s.  Windows of up to
// 8 vectors take an unrolled kernel (coefficients and pointers in registers,
// 16-byte moves); the general one serves the rest.
template <typename T, int K>
struct CombineKArgs {
    const T* q;
    CombinePtrs<T> ca;
    const double* coef;
    T* out;
    Seg g;
    int vec;
};
template <typename T, int K>
struct CombineKBody {
    static constexpr int kBlock = 256;
    using Args = CombineKArgs<T, K>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const T* __restrict__ q = args_.q;
        const CombinePtrs<T>& ca = args_.ca;
        const double* __restrict__ coef = args_.coef;
        T* __restrict__ out = args_.out;
        const Seg& g = args_.g;
        int vec = args_.vec;
        const int c = bk.y / g.nseg, s = bk.y % g.nseg;
        const long long base = c * g.cstride + s * g.seglen;
        T cs[K];
        const T* xk[K];
    #pragma unroll
        for (int k = 0; k < K; ++k) {
            cs[k] = T(coef[k * g.nseg + s]);
            xk[k] = ca.x[k] + base;
        }
        if (vec) {
            constexpr int W = Vec16<T>::W;
            const long long nv = g.seglen / W;
            const Vec16<T>* qv = reinterpret_cast<const Vec16<T>*>(q + base);
            Vec16<T>* ov = reinterpret_cast<Vec16<T>*>(out + base);
            for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < nv;
                 i += (long long)bk.gx * blockDim.x) {
                const Vec16<T> qi = qv[i];
                Vec16<T> xv[K];
    #pragma unroll
                for (int k = 0; k < K; ++k) xv[k] = reinterpret_cast<const Vec16<T>*>(xk[k])[i];
                Vec16<T> acc;
    #pragma unroll
                for (int w = 0; w < W; ++w) {
                    T a = qi.v[w];
    #pragma unroll
                    for (int k = 0; k < K; ++k) a += cs[k] * (qi.v[w] - xv[k].v[w]);
                    acc.v[w] = a;
                }
                ov[i] = acc;
            }
        } else {
            for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < g.seglen;
                 i += (long long)bk.gx * blockDim.x) {
                const T qi = q[base + i];
                T acc = qi;
    #pragma unroll
                for (int k = 0; k < K; ++k) acc += cs[k] * (qi - xk[k][i]);
                out[base + i] = acc;
            }
        }
    }
};

template <typename T>
struct CombineArgs {
    const T* q;
    CombinePtrs<T> ca;
    const double* coef;
    int K;
    T* out;
    Seg g;
};
template <typename T>
struct CombineBody {
    static constexpr int kBlock = 256;
    using Args = CombineArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const T* __restrict__ q = args_.q;
        const CombinePtrs<T>& ca = args_.ca;
        const double* __restrict__ coef = args_.coef;
        int K = args_.K;
        T* __restrict__ out = args_.out;
        const Seg& g = args_.g;
        const int c = bk.y / g.nseg, s = bk.y % g.nseg;
        const long long base = c * g.cstride + s * g.seglen;
        // the coefficients are read where they are used (wave-uniform
        // addresses, scalar loads): a per-thread array of them would live in
        // scratch memory
        for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < g.seglen;
             i += (long long)bk.gx * blockDim.x) {
            const T qi = q[base + i];
            T acc = qi;
            for (int k = 0; k < K; ++k) acc += T(coef[k * g.nseg + s]) * (qi - ca.x[k][base + i]);
            out[base + i] = acc;
        }
    }
};

// det of grad y = Id + (h_a dD_a/dx_b) from the d x d derivative fields
// J[a d + b] = dD_a/dx_b; per segment: max(-det), max(det), sum(det - 1),
// sum((det - 1)^2) (NaN counts as -inf / +inf for the extremes).
template <typename T>
struct DetArgs {
    const T* J[9];
    double h[3];
    int d;
};

template <typename T>
struct DetStatsArgs {
    DetArgs<T> a;
    Seg g;
    T* det;
    double* partial;
};
template <typename T>
struct DetStatsBody {
    static constexpr int kBlock = kRedThreads;
    using Args = DetStatsArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const DetArgs<T>& a = args_.a;
        const Seg& g = args_.g;
        T* det = args_.det;
        double* __restrict__ partial = args_.partial;
        __shared__ double sh[kRedThreads / 64];
        const int s = bk.y;
        double mn = -INFINITY, mx = -INFINITY, s1 = 0.0, s2 = 0.0;
        for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < g.seglen;
             i += (long long)bk.gx * blockDim.x) {
            const long long e = s * g.seglen + i;
            double m[3][3];
            for (int r = 0; r < a.d; ++r)
                for (int c = 0; c < a.d; ++c)
                    m[r][c] = (r == c ? 1.0 : 0.0) + a.h[r] * static_cast<double>(a.J[r * a.d + c][e]);
            const double dt = a.d == 2 ? m[0][0] * m[1][1] - m[0][1] * m[1][0]
                                       : m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
                                             m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                                             m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
            if (det) det[e] = static_cast<T>(dt);
            if (dt == dt) {
                mn = fmax(mn, -dt);
                mx = fmax(mx, dt);
                s1 += dt - 1.0;
                s2 += (dt - 1.0) * (dt - 1.0);
            } else {
                mn = mx = INFINITY;
                s1 = s2 = NAN;
            }
        }
        const double r0 = block_reduce<true>(mn, sh);
        const double r1 = block_reduce<true>(mx, sh);
        const double r2 = block_reduce<false>(s1, sh);
        const double r3 = block_reduce<false>(s2, sh);
        if (threadIdx.x == 0) {
            const long long nb = bk.gx, ns = bk.gy;
            partial[(0 * ns + s) * nb + bk.x] = r0;
            partial[(1 * ns + s) * nb + bk.x] = r1;
            partial[(2 * ns + s) * nb + bk.x] = r2;
            partial[(3 * ns + s) * nb + bk.x] = r3;
        }
    }
};

inline int stream_blocks(long long n) {
    long long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return static_cast<int>(b);
}

// blocks per row of a segment-wise vector update (rows = ncomp * nseg)
int row_blocks(const Seg& g) {
    const int rows = g.ncomp * g.nseg;
    int b = stream_blocks(g.seglen);
    if ((long long)b * rows > 8192) b = std::max(1, 8192 / rows);
    return b;
}

// blocks per segment for a reduction of nq quantities
int seg_blocks(const Seg& g, int nq) {
    long long b = reduction_blocks(g.ncomp * g.seglen);
    const long long cap = kPartialCap / ((long long)nq * g.nseg);
    if (b > cap) b = cap;
    return static_cast<int>(b < 1 ? 1 : b);
}

template <typename T, int K>
hipError_t gram_k(const T* const* vecs, const Seg& g, double* partial, double* res,
                  hipStream_t st) {
    VecList<T, K> vl;
    for (int a = 0; a < K; ++a) vl.p[a] = vecs[a];
    constexpr int NP = K * (K + 1) / 2;
    const int nb = seg_blocks(g, NP);
    bool vec = vec16_rows<T>(g, {});
    for (int a = 0; a < K; ++a) vec = vec && vec16_rows<T>(g, {vecs[a]});
    submit<GramBody<T, K>>(dim3(nb, g.nseg), 0, st, GramArgs<T, K>{vl, g, vec ? 1 : 0, partial});
    launch_finish<false>(partial, nb, NP * g.nseg, res, st);
    return hipGetLastError();
}

}  // namespace

int reduction_blocks(long long n) {
    long long b = (n + kRedThreads * 8 - 1) / (kRedThreads * 8);
    if (b > kMaxRedBlocks) b = kMaxRedBlocks;
    if (b < 1) b = 1;
    return static_cast<int>(b);
}

bool seg_valid(const Seg& g) {
    return g.nseg >= 1 && g.nseg <= kMaxSeg && g.ncomp >= 1 && g.seglen >= 1;
}

template <typename T>
hipError_t launch_sumsq_diff(const T* a, const T* b, T* lam, const Seg& g, double* partial,
                             double* res, hipStream_t st) {
    if (!seg_valid(g)) return hipErrorInvalidValue;
    const int nb = seg_blocks(g, 1);
    const int vec = vec16_rows<T>(g, {a, b, lam}) ? 1 : 0;
    submit<SumsqDiffBody<T>>(dim3(nb, g.nseg), 0, st, SumsqDiffArgs<T>{a, b, lam, g, vec, partial});
    launch_finish<false>(partial, nb, g.nseg, res, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dot(const T* a, const T* b, const Seg& g, double* partial, double* res,
                      hipStream_t st) {
    if (!seg_valid(g)) return hipErrorInvalidValue;
    const int nb = seg_blocks(g, 1);
    const int vec = vec16_rows<T>(g, {a, b}) ? 1 : 0;
    submit<DotBody<T>>(dim3(nb, g.nseg), 0, st, DotArgs<T>{a, b, g, vec, partial});
    launch_finish<false>(partial, nb, g.nseg, res, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_maxabs(const T* a, const Seg& g, double* partial, double* res, hipStream_t st) {
    if (!seg_valid(g)) return hipErrorInvalidValue;
    const int nb = seg_blocks(g, 1);
    const int vec = vec16_rows<T>(g, {a}) ? 1 : 0;
    submit<MaxabsBody<T>>(dim3(nb, g.nseg), 0, st, MaxabsArgs<T>{a, g, vec, partial});
    launch_finish<true>(partial, nb, g.nseg, res, st);
    return hipGetLastError();
}

// The packed Gram kernel writes the upper triangle in row order; the host
// unpacks.  res[q nseg + s] receives packed entry q of segment s.
template <typename T>
hipError_t launch_gram(const T* const* vecs, int K, const Seg& g, double* partial, double* res,
                       hipStream_t st) {
    if (!seg_valid(g)) return hipErrorInvalidValue;
    switch (K) {
        case 1: return gram_k<T, 1>(vecs, g, partial, res, st);
        case 2: return gram_k<T, 2>(vecs, g, partial, res, st);
        case 3: return gram_k<T, 3>(vecs, g, partial, res, st);
        case 4: return gram_k<T, 4>(vecs, g, partial, res, st);
        case 5: return gram_k<T, 5>(vecs, g, partial, res, st);
        case 6: return gram_k<T, 6>(vecs, g, partial, res, st);
        case 7: return gram_k<T, 7>(vecs, g, partial, res, st);
        case 8: return gram_k<T, 8>(vecs, g, partial, res, st);
        default: break;
    }
    if (K < 1 || K > kMaxGram) return hipErrorInvalidValue;
    // one pass over the K vectors; the partials of NP quantities per segment
    // must fit the caller's buffer (kGramPartialCap doubles)
    const long long NP = (long long)K * (K + 1) / 2;
    long long nb = reduction_blocks(g.ncomp * g.seglen);
    const long long cap = kGramPartialCap / (NP * g.nseg);
    if (cap < 1) return hipErrorInvalidValue;
    if (nb > cap) nb = cap;
    PtrList<T> pl{};
    for (int a = 0; a < K; ++a) pl.p[a] = vecs[a];
    const int Kp = 4 * ((K + 3) / 4);
    const size_t lds = sizeof(double) * std::max(Kp * kGramE, kRedThreads * 16);
    submit<GramBigBody<T>>(dim3((unsigned)nb, g.nseg), lds, st, GramBigArgs<T>{pl, K, g, partial});
    launch_finish<false>(partial, (int)nb,
                                                                      (int)(NP * g.nseg), res, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_det_stats(const T* const* J, const double* h, int d, const Seg& g, T* det,
                            double* partial, double* res, hipStream_t st) {
    if (!seg_valid(g) || (d != 2 && d != 3)) return hipErrorInvalidValue;
    DetArgs<T> a{};
    for (int q = 0; q < d * d; ++q) a.J[q] = J[q];
    for (int q = 0; q < 3; ++q) a.h[q] = q < d ? h[q] : 0.0;
    a.d = d;
    const int nb = seg_blocks(g, 4);
    submit<DetStatsBody<T>>(dim3(nb, g.nseg), 0, st, DetStatsArgs<T>{a, g, det, partial});
    launch_finish<true>(partial, nb, 2 * g.nseg, res, st);
    launch_finish<false>(partial + (long long)2 * g.nseg * nb, nb, 2 * g.nseg,
                                             res + 2 * g.nseg, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy(const T* a, const double* s, const T* b, T* out, const Seg& g,
                       hipStream_t st) {
    if (!seg_valid(g)) return hipErrorInvalidValue;
    SegCoef sc{};
    for (int i = 0; i < g.nseg; ++i) sc.c[i] = s[i];
    submit<AxpyBody<T>>(dim3(row_blocks(g), g.ncomp * g.nseg), 0, st, AxpyArgs<T>{a, sc, b, out, g});
    return hipGetLastError();
}

template <typename T>
hipError_t launch_outer(const T* g, const T* x, T* out, int d, long long n, hipStream_t st) {
    if (d < 1 || d > 3 || n < 1) return hipErrorInvalidValue;
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    submit<OuterBody<T>>(dim3((unsigned)blocks), 0, st, OuterArgs<T>{g, x, out, d, n});
    return hipGetLastError();
}

template <typename T>
hipError_t launch_combine(const T* q, const T* const* x, const double* coef, int K, T* out,
                          const Seg& g, hipStream_t st) {
    if (K < 0 || K > kMaxCombine || !seg_valid(g)) return hipErrorInvalidValue;
    CombinePtrs<T> ca;
    for (int k = 0; k < kMaxCombine; ++k) ca.x[k] = k < K ? x[k] : nullptr;
    const dim3 grid(row_blocks(g), g.ncomp * g.nseg);
    bool vec = vec16_rows<T>(g, {q, out});
    for (int k = 0; k < K; ++k) vec = vec && vec16_rows<T>(g, {x[k]});
    const int v = vec ? 1 : 0;
    switch (K) {
#define GAN_COMBINE(KK) \
    case KK: submit<CombineKBody<T, KK>>(dim3(grid), 0, st, CombineKArgs<T, KK>{q, ca, coef, out, g, v}); break;
        GAN_COMBINE(1)
        GAN_COMBINE(2)
        GAN_COMBINE(3)
        GAN_COMBINE(4)
        GAN_COMBINE(5)
        GAN_COMBINE(6)
        GAN_COMBINE(7)
        GAN_COMBINE(8)
#undef GAN_COMBINE
        default: submit<CombineBody<T>>(dim3(grid), 0, st, CombineArgs<T>{q, ca, coef, K, out, g});
    }
    return hipGetLastError();
}

#define GAN_INST(T)                                                                               \
    template hipError_t launch_sumsq_diff<T>(const T*, const T*, T*, const Seg&, double*, double*,  \
                                             hipStream_t);                                        \
    template hipError_t launch_dot<T>(const T*, const T*, const Seg&, double*, double*,           \
                                      hipStream_t);                                               \
    template hipError_t launch_maxabs<T>(const T*, const Seg&, double*, double*, hipStream_t);    \
    template hipError_t launch_gram<T>(const T* const*, int, const Seg&, double*, double*,        \
                                       hipStream_t);                                              \
    template hipError_t launch_axpy<T>(const T*, const double*, const T*, T*, const Seg&,         \
                                       hipStream_t);                                              \
    template hipError_t launch_combine<T>(const T*, const T* const*, const double*, int, T*,      \
                                          const Seg&, hipStream_t);                               \
    template hipError_t launch_outer<T>(const T*, const T*, T*, int, long long, hipStream_t);     \
    template hipError_t launch_det_stats<T>(const T* const*, const double*, int, const Seg&, T*,  \
                                            double*, double*, hipStream_t);
GAN_INST(float)
GAN_INST(double)
#undef GAN_INST

}  // namespace gan
