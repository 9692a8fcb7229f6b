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
#include <type_traits>

#include "fft_core.hpp"
#include "launch.hpp"
#include "group.hpp"
#include "reduce.hpp"

namespace gan {

// Dynamic LDS of the transform kernels (16-byte aligned for complex<double>).
extern __shared__ double2 gan_smem[];

namespace {

constexpr int kFftThreads = 256;
constexpr int kItems = 8;           // tile elements per thread (tile <= 2048 elements)
// Threads of the body-force derivative kernel: its tile of kItems reals per
// thread then spans 128 contiguous bytes of real pencils along the strided
// axes for lengths up to 128, and 64 up to 256 (with 256 threads: 64 and 32).
constexpr int kDerivThreads = 512;
// Complex axis passes of length >= kWideLength run 512-thread tiles (up to
// 80 KB of LDS), so that along the strided axes a tile spans 128 (256, 192)
// or 64 (384, 512) contiguous bytes instead of half that; shorter lengths keep
// 256 threads (their tiles already span 128 bytes).  The fused spectral pass
// keeps 256 threads at every length (its tiles hold every component: wider
// ones were slower).
constexpr int kWideLength = 192;
constexpr int kWideThreads = 512;
constexpr size_t kWideLds = 80 * 1024;
inline int c2c_threads(int L) { return L >= kWideLength ? kWideThreads : kFftThreads; }
constexpr int kMaxTime = 65;
constexpr int kLdsBudget = 64 * 1024;
constexpr int kTilesPerBlock = 2;  // grid-strided transforms: tiles per workgroup

// log2 of the complex pencils per tile for kernels whose tile holds 2 PC real
// pencils of length L (2 PC L <= kFftThreads * kItems), with two complex LDS
// buffers and the twiddle table within the LDS budget.
// Two padded buffers of PC L complex elements and the twiddle table.
size_t fft_lds_bytes(int PC, int L, int bytes_per_complex) {
    return (size_t)(2 * lpad_size(PC * L) + L) * bytes_per_complex;
}
int pc_shift_real(int L, int bytes_per_complex, long long npencils, int threads = kFftThreads) {
    int s = 0;
    while ((2 << (s + 1)) * L <= threads * kItems && (2LL << s) < npencils &&
           fft_lds_bytes(1 << (s + 1), L, bytes_per_complex) <= kLdsBudget &&
           s < (threads > kFftThreads ? 6 : 5))
        ++s;
    return s;
}
// pc_shift_real when the pencils are not the limit (every large grid), as a
// constant for the kernels compiled for it.
constexpr int pc_shift_real_full(int L, int bytes_per_complex, int threads) {
    int s = 0;
    while (true) {
        const long long n = (long long)(1 << (s + 1)) * L;
        const long long lds = (2 * (n + (n >> 4) + 1) + L) * (long long)bytes_per_complex;
        if (!((2 << (s + 1)) * L <= threads * kItems && lds <= (long long)kLdsBudget &&
              s < (threads > kFftThreads ? 6 : 5)))
            break;
        ++s;
    }
    return s;
}
// Same for in-place complex transforms: tiles of PC complex pencils.
int pc_shift_cplx(int L, int bytes_per_complex, long long npencils, int threads = kFftThreads) {
    const size_t budget = threads > kFftThreads ? kWideLds : kLdsBudget;
    int s = 0;
    while ((1 << (s + 1)) * L <= threads * kItems && (1LL << s) < npencils &&
           fft_lds_bytes(1 << (s + 1), L, bytes_per_complex) <= budget && s < 5)
        ++s;
    return s;
}

constexpr int pc_shift_cplx_full(int L, int bytes_per_complex, int threads = kFftThreads) {
    const long long budget = threads > kFftThreads ? (long long)kWideLds : (long long)kLdsBudget;
    int s = 0;
    while (true) {
        const long long n = (long long)(1 << (s + 1)) * L;
        const long long lds = (2 * (n + (n >> 4) + 1) + L) * (long long)bytes_per_complex;
        if (!((1 << (s + 1)) * L <= threads * kItems && lds <= budget && s < 5)) break;
        ++s;
    }
    return s;
}

// Pencils along `axis` of an (n0, n1, w) array (w = n2 for real data, n2/2+1
// for the half spectrum), numbered p = 0..count-1 so that consecutive pencils
// of the strided axes are adjacent in memory.
__host__ __device__ inline long long pencil_count(const Dims& dm, int axis, int w) {
    return axis == 2 ? (long long)dm.n[0] * dm.n[1]
                     : (axis == 1 ? (long long)dm.n[0] * w : (long long)dm.n[1] * w);
}
// (pencil counts are below 2^31: the division is done in 32 bits, which costs
// a tenth of the 64-bit sequence)
__device__ inline long long pencil_base(const Dims& dm, int axis, int w, long long p) {
    if (axis == 2) return p * w;
    if (axis == 1) {
        const unsigned up = static_cast<unsigned>(p), uw = static_cast<unsigned>(w);
        const unsigned q = up / uw;
        return (long long)q * dm.n[1] * w + (up - q * uw);
    }
    return p;
}
__device__ inline long long pencil_stride(const Dims& dm, int axis, int w) {
    return axis == 2 ? 1 : (axis == 1 ? w : (long long)dm.n[1] * w);
}

template <typename T, int NT = kFftThreads>
__device__ inline C2<T>* twiddles_to_lds(const FftPlan<T>& pl, C2<T>* tws) {
    for (int m = threadIdx.x; m < pl.L; m += NT) tws[m] = pl.tw[m];
    return tws;
}

// Transform of the tile: compiled for length LC when LC > 0 (with the
// constant log2 pencil count PCS when PCS >= 0), else driven by the runtime
// plan.
template <typename T, int LC, int NT = kFftThreads, int PCS = -1>
__device__ inline C2<T>* tile_fft(C2<T>* a, C2<T>* b, const FftPlan<T>& pl, const C2<T>* tw,
                                  int pcshift, int dir) {
    if constexpr (LC > 0)
        return block_fft_ct<T, LC, NT, 0, 1, false, PCS>(a, b, tw, pcshift, dir);
    else
        return block_fft<T>(a, b, pl, tw, pcshift, dir);
}

// Lengths with compiled transforms (the grid sizes of the workloads); any
// other 2^a 3^b length takes the runtime plan.
template <typename F>
void with_length(int L, F&& f) {
    switch (L) {
        case 32: f(std::integral_constant<int, 32>{}); break;
        case 64: f(std::integral_constant<int, 64>{}); break;
        case 96: f(std::integral_constant<int, 96>{}); break;
        case 128: f(std::integral_constant<int, 128>{}); break;
        case 192: f(std::integral_constant<int, 192>{}); break;
        case 256: f(std::integral_constant<int, 256>{}); break;
        case 384: f(std::integral_constant<int, 384>{}); break;
        case 512: f(std::integral_constant<int, 512>{}); break;
        default: f(std::integral_constant<int, 0>{}); break;
    }
}

// The same choice on the device, for the bodies of merged launches whose
// classes have different lengths.  Only the compiled lengths merge (the
// runtime-plan body keeps its arrays in scratch once inlined beside the
// others), so the host submits other lengths as families of their own.
template <typename F>
__device__ __forceinline__ void with_length_dev(int L, F&& f) {
    switch (L) {
        case 32: f(std::integral_constant<int, 32>{}); break;
        case 64: f(std::integral_constant<int, 64>{}); break;
        case 96: f(std::integral_constant<int, 96>{}); break;
        case 128: f(std::integral_constant<int, 128>{}); break;
        case 192: f(std::integral_constant<int, 192>{}); break;
        case 256: f(std::integral_constant<int, 256>{}); break;
        case 384: f(std::integral_constant<int, 384>{}); break;
        case 512: f(std::integral_constant<int, 512>{}); break;
        default: break;
    }
}
// The merged family of a length: its Any body for a compiled length, the
// length's own body otherwise.
template <int LC, class Body, class AnyBody>
using MergeFamily = typename std::conditional<LC == 0, Body, AnyBody>::type;

// Item e of a tile of NP real pencils x L: its pencil r and position i.
// Strided axes put the pencil index fastest (coalesced over adjacent
// pencils); the contiguous axis puts the position fastest.
__device__ inline void item_pos(int axis, int q, int L, int npshift, int& r, int& i) {
    if (axis != 2) {
        r = q & ((1 << npshift) - 1);
        i = q >> npshift;
    } else {
        r = q / L;
        i = q - r * L;
    }
}

template <typename T, int MT>
struct DerivArgs {
    Dims dm;
    FftPlan<T> pl;
    int axis, pcshift;
    int ntime;
    int accumulate;
    int has_g;
    T* out;
    const T* F[MT];
    const T* G[MT];
    double w[MT];
};
// Launches with at most kGroupTime time levels carry the short argument list
// (small enough to merge the launches of a group handle's classes).
constexpr int kGroupTime = 9;

// out = [out +] sum_t w_t G_t d/dx_axis F_t over one tile of 2 PC real pencils.
// The loads of G_t and F_{t+1} are issued before the transforms of step t so
// that they complete while the LDS passes run.  PCS >= 0 (compiled lengths
// only): the tile's log2 pencil count a.pcshift is known to equal PCS, and
// the transforms' LDS addressing is compiled for it.
template <typename T, int LC, int MT, int PCS = -1>
struct DerivAxisBody {
    static_assert(PCS < 0 || LC > 0, "a constant pencil count needs a compiled length");
    static constexpr int kBlock = kDerivThreads;
    using Args = DerivArgs<T, MT>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const DerivArgs<T, MT>& a = args_;
        const int L = LC > 0 ? LC : a.pl.L;
        const int pcs = PCS >= 0 ? PCS : a.pcshift;
        const int PC = 1 << pcs;
        const int npshift = pcs + 1;
        C2<T>* bufA = reinterpret_cast<C2<T>*>(gan_smem);
        C2<T>* bufB = bufA + lpad_size(PC * L);
        const FftPlan<T>& pl = a.pl;
        const C2<T>* tw = twiddles_to_lds<T, kDerivThreads>(a.pl, bufB + lpad_size(PC * L));
        const Dims& dm = a.dm;
        const long long npen = pencil_count(dm, a.axis, dm.n[2]);
        const long long stride = pencil_stride(dm, a.axis, dm.n[2]);
        const long long p0 = (long long)bk.x << npshift;
        const int nitems = (2 * PC) * L;
        const T inv_l = T(1) / T(L);

        long long off[kItems];
        int slot[kItems];  // T index in bufA: 2 * complex index + (0 real | 1 imag); -1: no item
        bool ok[kItems];
        T acc[kItems], fv[kItems], gv[kItems];
    #pragma unroll
        for (int e = 0; e < kItems; ++e) {
            const int q = threadIdx.x + e * kDerivThreads;
            slot[e] = -1;
            ok[e] = false;
            off[e] = 0;
            if (q < nitems) {
                int r, i;
                item_pos(a.axis, q, L, npshift, r, i);
                slot[e] = 2 * lpad((i << pcs) + (r & (PC - 1))) + (r >> pcs);
                ok[e] = p0 + r < npen;
                if (ok[e]) off[e] = pencil_base(dm, a.axis, dm.n[2], p0 + r) + i * stride;
            }
            acc[e] = (ok[e] && a.accumulate) ? a.out[off[e]] : T(0);
            fv[e] = ok[e] ? a.F[0][off[e]] : T(0);
            gv[e] = T(1);
        }
        T* flat = reinterpret_cast<T*>(bufA);
        for (int t = 0; t < a.ntime; ++t) {
    #pragma unroll
            for (int e = 0; e < kItems; ++e)
                if (slot[e] >= 0) flat[slot[e]] = fv[e];
            __syncthreads();
            const T* G = a.has_g ? a.G[t] : nullptr;
            const bool more = t + 1 < a.ntime;
            const T* Fn = more ? a.F[t + 1] : nullptr;
    #pragma unroll
            for (int e = 0; e < kItems; ++e) {
                if (G) gv[e] = ok[e] ? G[off[e]] : T(0);
                if (more) fv[e] = ok[e] ? Fn[off[e]] : T(0);
            }
            C2<T>* X;
            if constexpr (LC > 0) {
                // the derivative factor is applied by the last forward stage
                X = block_fft_ct<T, LC, kDerivThreads, 0, 1, true, PCS>(bufA, bufB, tw, pcs, -1, inv_l);
            } else {
                X = tile_fft<T, LC, kDerivThreads>(bufA, bufB, pl, tw, a.pcshift, -1);
                for (int q = threadIdx.x; q < PC * L; q += kDerivThreads) {
                    const int i = q >> a.pcshift;
                    X[lpad(q)] = cmuli(X[lpad(q)], T(wavenumber_odd(i, L)) * inv_l);
                }
                __syncthreads();
            }
            const C2<T>* Y = tile_fft<T, LC, kDerivThreads, PCS>(X, X == bufA ? bufB : bufA, pl, tw, pcs, +1);
            const T* yflat = reinterpret_cast<const T*>(Y);
            const T wt = T(a.w[t]);
    #pragma unroll
            for (int e = 0; e < kItems; ++e)
                if (ok[e]) acc[e] += wt * gv[e] * yflat[slot[e]];
            __syncthreads();
        }
    #pragma unroll
        for (int e = 0; e < kItems; ++e)
            if (ok[e]) a.out[off[e]] = acc[e];
    }
};

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
struct R2cRowsArgs {
    Dims dm;
    FftPlan<TC> pl0;
    int pcshift;
    InPtrs<TI> ip;
    SpecPtrs<TC> sp;
};
template <typename TI, typename TC, int LC, int PCS = -1>
struct R2cRowsBody {
    static constexpr int kBlock = kFftThreads;
    using Args = R2cRowsArgs<TI, TC>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const FftPlan<TC>& pl0 = args_.pl0;
        const int pcshift = PCS >= 0 ? PCS : args_.pcshift;
        const InPtrs<TI>& ip = args_.ip;
        const SpecPtrs<TC>& sp = args_.sp;
        using T = TC;
        const int L = LC > 0 ? LC : pl0.L;
        const int PC = 1 << pcshift;
        C2<T>* bufA = reinterpret_cast<C2<T>*>(gan_smem);
        C2<T>* bufB = bufA + lpad_size(PC * L);
        const FftPlan<T>& pl = pl0;
        const C2<T>* tw = twiddles_to_lds(pl0, bufB + lpad_size(PC * L));
        const TI* in = ip.in[bk.y];
        C2<T>* spec = sp.spec[bk.y];
        const long long rows = (long long)dm.n[0] * dm.n[1];
        const long long q0 = (long long)bk.x * 2 * PC;
        const int nitems = 2 * PC * L;
        T* flat = reinterpret_cast<T*>(bufA);
        // rows of a compiled length that is a multiple of 16 bytes move with
        // 16-byte loads, WI consecutive elements per thread
        constexpr int WI = 16 / (int)sizeof(TI);
        if (LC > 0 && LC % WI == 0 && (reinterpret_cast<unsigned long long>(in) & 15) == 0) {
            struct alignas(16) V {
                TI x[WI];
            };
            V vals[kItems / WI];
    #pragma unroll
            for (int e = 0; e < kItems / WI; ++e) {
                const int q = (threadIdx.x + e * kFftThreads) * WI;
                const int r = q / L, i = q - r * L;
                if (q < nitems && q0 + r < rows) {
                    vals[e] = *reinterpret_cast<const V*>(in + (q0 + r) * L + i);
                } else {
    #pragma unroll
                    for (int w = 0; w < WI; ++w) vals[e].x[w] = TI(0);
                }
            }
    #pragma unroll
            for (int e = 0; e < kItems / WI; ++e) {
                const int q = (threadIdx.x + e * kFftThreads) * WI;
                if (q < nitems) {
                    const int r = q / L, i = q - r * L;
    #pragma unroll
                    for (int w = 0; w < WI; ++w)
                        flat[2 * lpad(((i + w) << pcshift) + (r & (PC - 1))) + (r >> pcshift)] =
                            T(vals[e].x[w]);
                }
            }
        } else {
            T vals[kItems];
    #pragma unroll
            for (int e = 0; e < kItems; ++e) {
                const int q = threadIdx.x + e * kFftThreads;
                const int r = q / L, i = q - r * L;
                vals[e] = (q < nitems && q0 + r < rows) ? T(in[(q0 + r) * L + i]) : T(0);
            }
    #pragma unroll
            for (int e = 0; e < kItems; ++e) {
                const int q = threadIdx.x + e * kFftThreads;
                if (q < nitems) {
                    const int r = q / L, i = q - r * L;
                    flat[2 * lpad((i << pcshift) + (r & (PC - 1))) + (r >> pcshift)] = vals[e];
                }
            }
        }
        __syncthreads();
        const C2<T>* Z = tile_fft<T, LC, kFftThreads, PCS>(bufA, bufB, pl, tw, pcshift, -1);
        const int nh = dm.n2h;
        for (int q = threadIdx.x; q < 2 * PC * nh; q += kFftThreads) {
            const int r = q / nh, k = q - r * nh;
            if (q0 + r >= rows) continue;
            const int p = r & (PC - 1);
            const C2<T> zk = Z[lpad((k << pcshift) + p)];
            const int km = k == 0 ? 0 : L - k;
            const C2<T> zm = Z[lpad((km << pcshift) + p)];
            C2<T> o;
            if ((r >> pcshift) == 0) o = cmk(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));
            else o = cmk(T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x));
            spec[(q0 + r) * nh + k] = o;
        }
    }
};

// In-place complex transform of the half spectrum along axis 0 or 1, on tiles
// of PC adjacent pencils.
template <typename T>
struct C2cAxisArgs {
    Dims dm;
    FftPlan<T> pl0;
    int axis;
    int pcshift;
    int dir;
    SpecPtrs<T> sp;
};
template <typename T, int LC, int NT = kFftThreads, int PCS = -1>
struct C2cAxisBody {
    static constexpr int kBlock = NT;
    using Args = C2cAxisArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const FftPlan<T>& pl0 = args_.pl0;
        int axis = args_.axis;
        const int pcshift = PCS >= 0 ? PCS : args_.pcshift;
        int dir = args_.dir;
        const SpecPtrs<T>& sp = args_.sp;
        const int L = LC > 0 ? LC : pl0.L;
        const int PC = 1 << pcshift;
        C2<T>* bufA = reinterpret_cast<C2<T>*>(gan_smem);
        C2<T>* bufB = bufA + lpad_size(PC * L);
        const FftPlan<T>& pl = pl0;
        const C2<T>* tw = twiddles_to_lds<T, NT>(pl0, bufB + lpad_size(PC * L));
        C2<T>* spec = sp.spec[bk.y];
        const int nh = dm.n2h;
        const long long npen = pencil_count(dm, axis, nh);
        const long long stride = pencil_stride(dm, axis, nh);
        const long long ntiles = (npen + PC - 1) >> pcshift;
        const int pl_ = threadIdx.x & (PC - 1);
        const int nitems = PC * L;
        // Tiles of PC adjacent pencils, grid-strided over the workgroups; the next
        // tile's data is loaded into registers while the current one transforms.
        auto load = [&](long long tile, C2<T>* vals, long long& base, bool& ok) {
            const long long p = (tile << pcshift) + pl_;
            ok = p < npen;
            base = ok ? pencil_base(dm, axis, nh, p) : 0;
    #pragma unroll
            for (int e = 0; e < kItems; ++e) {
                const int q = threadIdx.x + e * NT;
                vals[e] = (q < nitems && ok) ? spec[base + (q >> pcshift) * stride] : cmk(T(0), T(0));
            }
        };
        long long tile = bk.x;
        if (tile >= ntiles) return;
        C2<T> vals[kItems];
        long long base;
        bool ok;
        load(tile, vals, base, ok);
        for (;;) {
    #pragma unroll
            for (int e = 0; e < kItems; ++e) {
                const int q = threadIdx.x + e * NT;
                if (q < nitems) bufA[lpad(q)] = vals[e];
            }
            __syncthreads();
            const long long next = tile + bk.gx;
            long long nbase = 0;
            bool nok = false;
            if (next < ntiles) load(next, vals, nbase, nok);
            const C2<T>* Z = tile_fft<T, LC, NT, PCS>(bufA, bufB, pl, tw, pcshift, dir);
    #pragma unroll
            for (int e = 0; e < kItems; ++e) {
                const int q = threadIdx.x + e * NT;
                if (q < nitems && ok) spec[base + (q >> pcshift) * stride] = Z[lpad(q)];
            }
            if (next >= ntiles) break;
            __syncthreads();  // every thread has read Z before bufA is refilled
            tile = next;
            base = nbase;
            ok = nok;
        }
    }
};

// Workgroups for a grid-strided transform of `tiles` tiles per field: about
// `per` tiles each, so that the prefetch of the next tile has a tile to
// overlap with.
inline unsigned strided_blocks(long long tiles, int per) {
    long long b = (tiles + per - 1) / per;
    return (unsigned)(b < 1 ? 1 : b);
}

// Half-spectrum rows -> real rows: out = scale * x [+ add].
template <typename T>
struct C2rRowsArgs {
    Dims dm;
    FftPlan<T> pl0;
    int pcshift;
    T scale;
    SpecPtrs<T> sp;
    OutPtrs<T> op;
};
template <typename T, int LC, int PCS = -1>
struct C2rRowsBody {
    static constexpr int kBlock = kFftThreads;
    using Args = C2rRowsArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const FftPlan<T>& pl0 = args_.pl0;
        const int pcshift = PCS >= 0 ? PCS : args_.pcshift;
        T scale = args_.scale;
        const SpecPtrs<T>& sp = args_.sp;
        const OutPtrs<T>& op = args_.op;
        const int L = LC > 0 ? LC : pl0.L;
        const int PC = 1 << pcshift;
        C2<T>* bufA = reinterpret_cast<C2<T>*>(gan_smem);
        C2<T>* bufB = bufA + lpad_size(PC * L);
        const FftPlan<T>& pl = pl0;
        const C2<T>* tw = twiddles_to_lds(pl0, bufB + lpad_size(PC * L));
        const C2<T>* spec = sp.spec[bk.y];
        T* out = op.out[bk.y];
        const T* add = op.add[bk.y];
        const long long rows = (long long)dm.n[0] * dm.n[1];
        const long long q0 = (long long)bk.x * 2 * PC;
        const int nh = dm.n2h;
        const int nitems = PC * L;
        constexpr int EH = kItems / 2;  // PC L <= kFftThreads * kItems / 2
        C2<T> A[EH], B[EH];
    #pragma unroll
        for (int e = 0; e < EH; ++e) {
            const int q = threadIdx.x + e * kFftThreads;
            const int p = q / L, i = q - p * L;
            const int ks = 2 * i > L ? L - i : i;
            A[e] = (q < nitems && q0 + p < rows) ? spec[(q0 + p) * nh + ks] : cmk(T(0), T(0));
            B[e] = (q < nitems && q0 + p + PC < rows) ? spec[(q0 + p + PC) * nh + ks] : cmk(T(0), T(0));
        }
    #pragma unroll
        for (int e = 0; e < EH; ++e) {
            const int q = threadIdx.x + e * kFftThreads;
            if (q >= nitems) continue;
            const int p = q / L, i = q - p * L;
            const bool upper = 2 * i > L;
            const int ks = upper ? L - i : i;
            C2<T> a = A[e], b = B[e];
            if (ks == 0 || 2 * ks == L) {
                a.y = T(0);
                b.y = T(0);
            }
            if (upper) {
                a.y = -a.y;
                b.y = -b.y;
            }
            bufA[lpad((i << pcshift) + p)] = cmk(a.x - b.y, a.y + b.x);
        }
        __syncthreads();
        const C2<T>* Z = tile_fft<T, LC, kFftThreads, PCS>(bufA, bufB, pl, tw, pcshift, +1);
        constexpr int W = 16 / (int)sizeof(T);
        if (LC > 0 && LC % W == 0 && (reinterpret_cast<unsigned long long>(out) & 15) == 0 &&
            (reinterpret_cast<unsigned long long>(add) & 15) == 0) {
            // 16-byte stores (and loads of add), W consecutive elements per thread
            struct alignas(16) V {
                T x[W];
            };
            V addv[kItems / W];
    #pragma unroll
            for (int e = 0; e < kItems / W; ++e) {
                const int q = (threadIdx.x + e * kFftThreads) * W;
                const int r = q / L, i = q - r * L;
                if (add && q < 2 * nitems && q0 + r < rows) {
                    addv[e] = *reinterpret_cast<const V*>(add + (q0 + r) * L + i);
                } else {
    #pragma unroll
                    for (int w = 0; w < W; ++w) addv[e].x[w] = T(0);
                }
            }
    #pragma unroll
            for (int e = 0; e < kItems / W; ++e) {
                const int q = (threadIdx.x + e * kFftThreads) * W;
                const int r = q / L, i = q - r * L;
                if (q >= 2 * nitems || q0 + r >= rows) continue;
                V o;
    #pragma unroll
                for (int w = 0; w < W; ++w) {
                    const C2<T> z = Z[lpad(((i + w) << pcshift) + (r & (PC - 1)))];
                    o.x[w] = scale * ((r >> pcshift) ? z.y : z.x) + addv[e].x[w];
                }
                *reinterpret_cast<V*>(out + (q0 + r) * L + i) = o;
            }
            return;
        }
        T addv[kItems];
    #pragma unroll
        for (int e = 0; e < kItems; ++e) {
            const int q = threadIdx.x + e * kFftThreads;
            const int r = q / L, i = q - r * L;
            addv[e] = (add && q < 2 * nitems && q0 + r < rows) ? add[(q0 + r) * L + i] : T(0);
        }
    #pragma unroll
        for (int e = 0; e < kItems; ++e) {
            const int q = threadIdx.x + e * kFftThreads;
            const int r = q / L, i = q - r * L;
            if (q >= 2 * nitems || q0 + r >= rows) continue;
            const C2<T> z = Z[lpad((i << pcshift) + (r & (PC - 1)))];
            out[(q0 + r) * L + i] = scale * ((r >> pcshift) ? z.y : z.x) + addv[e];
        }
    }
};

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
    // 2-D: axis 0 stacks independent problems and carries no wavenumber
    const int k0 = dm.dim == 3 ? wavenumber(i0, dm.n[0]) : 0;
    const int k1 = wavenumber(i1, dm.n[1]), k2 = i2;
    kv.k2 = double(k0) * k0 + double(k1) * k1 + double(k2) * k2;
    kv.kt[0] = dm.dim == 3 ? wavenumber_odd(i0, dm.n[0]) : 0.0;
    kv.kt[1] = wavenumber_odd(i1, dm.n[1]);
    kv.kt[2] = (2 * i2 == dm.n[2]) ? 0.0 : double(i2);
    return kv;
}

// Stacked problems (2-D batches): number of them and the one holding
// half-spectrum element lin.
__host__ __device__ inline int spec_nseg(const Dims& dm) { return dm.dim == 2 ? dm.n[0] : 1; }
__device__ inline int spec_seg(const Dims& dm, long long lin) {
    return dm.dim == 2 ? (int)(lin / ((long long)dm.n[1] * dm.n2h)) : 0;
}
__device__ inline double seg_alpha(const SpecOpParams& sp, const Dims& dm, long long lin) {
    return sp.alpha_seg ? sp.alpha_seg[spec_seg(dm, lin)] : sp.alpha;
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
        // component c lies along internal axis c (3-D) or c + 1 (2-D); both
        // indices are constants here, so kt stays in registers
        const double k3 = kv.kt[c], k2 = c + 1 < 3 ? kv.kt[c + 1 < 3 ? c + 1 : 2] : 0.0;
        kc[c] = c < dim ? (dim == 3 ? k3 : k2) : 0.0;
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
struct SpecGradientArgs {
    Dims dm;
    SpecOpParams sp;
    SpecPtrs<double> vh;
    SpecPtrs<T> bh;
    SpecPtrs<T> gh;
};
template <typename T>
struct SpecGradientBody {
    static constexpr int kBlock = 256;
    using Args = SpecGradientArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const SpecOpParams& sp = args_.sp;
        const SpecPtrs<double>& vh = args_.vh;
        const SpecPtrs<T>& bh = args_.bh;
        const SpecPtrs<T>& gh = args_.gh;
        for (long long lin = bk.x * (long long)blockDim.x + threadIdx.x; lin < dm.NH;
             lin += (long long)bk.gx * blockDim.x) {
            const KVec kv = kvec(dm, lin);
            const double al = seg_alpha(sp, dm, lin) * ipow(kv.k2, sp.p);
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
};

template <typename T>
struct SpecPrecondArgs {
    Dims dm;
    SpecOpParams sp;
    SpecPtrs<T> gh;
    SpecPtrs<T> sh;
    SpecPtrs<T> keep;
    int has_keep;
};
template <typename T>
struct SpecPrecondBody {
    static constexpr int kBlock = 256;
    using Args = SpecPrecondArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const SpecOpParams& sp = args_.sp;
        const SpecPtrs<T>& gh = args_.gh;
        const SpecPtrs<T>& sh = args_.sh;
        const SpecPtrs<T>& keep = args_.keep;
        int has_keep = args_.has_keep;
        for (long long lin = bk.x * (long long)blockDim.x + threadIdx.x; lin < dm.NH;
             lin += (long long)bk.gx * blockDim.x) {
            const KVec kv = kvec(dm, lin);
            double l = ipow(kv.k2, sp.p);
            if (l == 0.0) l = 1.0;
            const T f = T(-1.0 / (seg_alpha(sp, dm, lin) * l));
            C2<T> g[3];
    #pragma unroll
            for (int c = 0; c < 3; ++c) g[c] = c < sp.dim ? gh.spec[c][lin] : cmk(T(0), T(0));
            if (sp.leray) leray_point(kv, sp.dim, g);
    #pragma unroll
            for (int c = 0; c < 3; ++c)
                if (c < sp.dim) {
                    const C2<T> z = cscale(g[c], f);
                    sh.spec[c][lin] = z;
                    if (has_keep) keep.spec[c][lin] = z;
                }
        }
    }
};

// The last forward and the first inverse pass of the complex transforms along
// `axis`, with a spectral operator in between, on tiles of PC pencils holding
// every component: per component the tile is transformed in LDS and kept in
// registers, the operator (which couples the components through the Leray
// projection) runs on the registers, and each component is transformed back
// and stored in place.  The transforms and the operator are the ones of
// c2c_axis_kernel and spec_gradient_kernel / spec_precond_kernel, so the
// result is bitwise that of the three separate passes, without the two
// round trips of the spectra through HBM between them.
template <typename T>
struct C2cSpecArgs {
    Dims dm;
    FftPlan<T> pl0;
    int axis;
    int pcshift;
    SpecOpParams sop;
    SpecPtrs<T> io;
    SpecPtrs<double> vh;
    SpecPtrs<T> keep;
    int has_keep;
    SpecPtrs<T> pre;  // kSpecGrad with has_keep: second copy of the direction's spectrum
};
template <typename T, int LC, int OP, int PCS = -1>
struct C2cSpecBody {
    static constexpr int kBlock = kFftThreads;
    using Args = C2cSpecArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const FftPlan<T>& pl0 = args_.pl0;
        int axis = args_.axis;
        const int pcshift = PCS >= 0 ? PCS : args_.pcshift;
        const SpecOpParams& sop = args_.sop;
        const SpecPtrs<T>& io = args_.io;
        const SpecPtrs<double>& vh = args_.vh;
        const SpecPtrs<T>& keep = args_.keep;
        int has_keep = args_.has_keep;
        const SpecPtrs<T>& pre = args_.pre;
        const int L = LC > 0 ? LC : pl0.L;
        const int PC = 1 << pcshift;
        C2<T>* bufA = reinterpret_cast<C2<T>*>(gan_smem);
        C2<T>* bufB = bufA + lpad_size(PC * L);
        const FftPlan<T>& pl = pl0;
        const C2<T>* tw = twiddles_to_lds(pl0, bufB + lpad_size(PC * L));
        const int nh = dm.n2h;
        const long long npen = pencil_count(dm, axis, nh);
        const long long stride = pencil_stride(dm, axis, nh);
        const long long ntiles = (npen + PC - 1) >> pcshift;
        const int pl_ = threadIdx.x & (PC - 1);
        const int nitems = PC * L;
        const int dim = sop.dim;
        for (long long tile = bk.x; tile < ntiles; tile += bk.gx) {
            const long long p = (tile << pcshift) + pl_;
            const bool ok = p < npen;
            const long long base = ok ? pencil_base(dm, axis, nh, p) : 0;
            C2<T> R[3][kItems];
    #pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c >= dim) break;
                const C2<T>* src = io.spec[c];
    #pragma unroll
                for (int e = 0; e < kItems; ++e) {
                    const int q = threadIdx.x + e * kFftThreads;
                    if (q < nitems)
                        bufA[lpad(q)] = ok ? src[base + (q >> pcshift) * stride] : cmk(T(0), T(0));
                }
                __syncthreads();
                const C2<T>* Z = tile_fft<T, LC, kFftThreads, PCS>(bufA, bufB, pl, tw, pcshift, -1);
    #pragma unroll
                for (int e = 0; e < kItems; ++e) {
                    const int q = threadIdx.x + e * kFftThreads;
                    R[c][e] = q < nitems ? Z[lpad(q)] : cmk(T(0), T(0));
                }
                __syncthreads();
            }
    #pragma unroll
            for (int e = 0; e < kItems; ++e) {
                const int q = threadIdx.x + e * kFftThreads;
                if (q >= nitems || !ok) continue;
                const long long lin = base + (q >> pcshift) * stride;
                const KVec kv = kvec(dm, lin);
                C2<T> g[3];
    #pragma unroll
                for (int c = 0; c < 3; ++c) g[c] = c < dim ? R[c][e] : cmk(T(0), T(0));
                if (sop.leray) leray_point(kv, dim, g);
                if constexpr (OP == kSpecGrad) {
                    const double al = seg_alpha(sop, dm, lin) * ipow(kv.k2, sop.p);
    #pragma unroll
                    for (int c = 0; c < 3; ++c)
                        if (c < dim) {
                            const C2<double> z = vh.spec[c][lin];
                            R[c][e] = cmk(T(al * z.x + double(g[c].x)), T(al * z.y + double(g[c].y)));
                        }
                    if (has_keep) {
                        // the next direction from this gradient's spectrum: the
                        // preconditioner below, applied to g^ instead of to the
                        // transform of the gradient once it is back on the grid
                        C2<T> h[3];
    #pragma unroll
                        for (int c = 0; c < 3; ++c) h[c] = c < dim ? R[c][e] : cmk(T(0), T(0));
                        if (sop.leray) leray_point(kv, dim, h);
                        double l = ipow(kv.k2, sop.p);
                        if (l == 0.0) l = 1.0;
                        const T f = T(-1.0 / (seg_alpha(sop, dm, lin) * l));
    #pragma unroll
                        for (int c = 0; c < 3; ++c)
                            if (c < dim) {
                                const C2<T> sv = cscale(h[c], f);
                                keep.spec[c][lin] = sv;
                                pre.spec[c][lin] = sv;
                            }
                    }
                } else {
                    double l = ipow(kv.k2, sop.p);
                    if (l == 0.0) l = 1.0;
                    const T f = T(-1.0 / (seg_alpha(sop, dm, lin) * l));
    #pragma unroll
                    for (int c = 0; c < 3; ++c)
                        if (c < dim) {
                            R[c][e] = cscale(g[c], f);
                            if (has_keep) keep.spec[c][lin] = R[c][e];
                        }
                }
            }
    #pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c >= dim) break;
    #pragma unroll
                for (int e = 0; e < kItems; ++e) {
                    const int q = threadIdx.x + e * kFftThreads;
                    if (q < nitems) bufA[lpad(q)] = R[c][e];
                }
                __syncthreads();
                const C2<T>* Z = tile_fft<T, LC, kFftThreads, PCS>(bufA, bufB, pl, tw, pcshift, +1);
                C2<T>* dst = io.spec[c];
    #pragma unroll
                for (int e = 0; e < kItems; ++e) {
                    const int q = threadIdx.x + e * kFftThreads;
                    if (q < nitems && ok) dst[base + (q >> pcshift) * stride] = Z[lpad(q)];
                }
                __syncthreads();
            }
        }
    }
};

// Bodies of merged launches: the transform length of each class is read from
// its plan and dispatched to the body compiled for it.
template <typename T, int MT>
struct DerivAxisAnyBody {
    static constexpr int kBlock = kDerivThreads;
    using Args = DerivArgs<T, MT>;
    __device__ __forceinline__ static void run(const Args& a, const Blk& bk) {
        with_length_dev(a.pl.L, [&](auto lc) __attribute__((always_inline)) { DerivAxisBody<T, decltype(lc)::value, MT>::run(a, bk); });
    }
};
template <typename TI, typename TC>
struct R2cRowsAnyBody {
    static constexpr int kBlock = kFftThreads;
    using Args = R2cRowsArgs<TI, TC>;
    __device__ __forceinline__ static void run(const Args& a, const Blk& bk) {
        with_length_dev(a.pl0.L, [&](auto lc) __attribute__((always_inline)) { R2cRowsBody<TI, TC, decltype(lc)::value>::run(a, bk); });
    }
};
template <typename T, int NT = kFftThreads>
struct C2cAxisAnyBody {
    static constexpr int kBlock = NT;
    using Args = C2cAxisArgs<T>;
    __device__ __forceinline__ static void run(const Args& a, const Blk& bk) {
        with_length_dev(a.pl0.L, [&](auto lc) __attribute__((always_inline)) { C2cAxisBody<T, decltype(lc)::value, NT>::run(a, bk); });
    }
};
template <typename T>
struct C2rRowsAnyBody {
    static constexpr int kBlock = kFftThreads;
    using Args = C2rRowsArgs<T>;
    __device__ __forceinline__ static void run(const Args& a, const Blk& bk) {
        with_length_dev(a.pl0.L, [&](auto lc) __attribute__((always_inline)) { C2rRowsBody<T, decltype(lc)::value>::run(a, bk); });
    }
};
template <typename T, int OP>
struct C2cSpecAnyBody {
    static constexpr int kBlock = kFftThreads;
    using Args = C2cSpecArgs<T>;
    __device__ __forceinline__ static void run(const Args& a, const Blk& bk) {
        with_length_dev(a.pl0.L, [&](auto lc) __attribute__((always_inline)) { C2cSpecBody<T, decltype(lc)::value, OP>::run(a, bk); });
    }
};

// The coarse space of the two-level preconditioner on a grid of c_i cells per
// axis: the wavenumbers |k_i| <= c_i/2 - 1 (the Nyquist modes, and for an odd
// c_i the top pair, dropped, so that restriction and prolongation are exact
// inverses on it).
__device__ inline bool coarse_kept(int k, int c) { return 2 * (k < 0 ? -k : k) <= c - 2; }

// sh[c] = sign (alpha lbar_p)^expo P gh[c]; with band_cut the modes outside
// the coarse space of this grid are set to zero.
template <typename T>
struct SpecPowArgs {
    Dims dm;
    SpecOpParams sp;
    SpecPtrs<T> gh;
    SpecPtrs<T> sh;
    double expo;
    double sign;
    int band_cut;
};
template <typename T>
struct SpecPowBody {
    static constexpr int kBlock = 256;
    using Args = SpecPowArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const SpecOpParams& sp = args_.sp;
        const SpecPtrs<T>& gh = args_.gh;
        const SpecPtrs<T>& sh = args_.sh;
        double expo = args_.expo;
        double sign = args_.sign;
        int band_cut = args_.band_cut;
        for (long long lin = bk.x * (long long)blockDim.x + threadIdx.x; lin < dm.NH;
             lin += (long long)bk.gx * blockDim.x) {
            const int i2 = (int)(lin % dm.n2h);
            const long long rest = lin / dm.n2h;
            const int i1 = (int)(rest % dm.n[1]), i0 = (int)(rest / dm.n[1]);
            const int k0 = dm.dim == 3 ? wavenumber(i0, dm.n[0]) : 0;
            const bool kept = (dm.dim == 2 || coarse_kept(k0, dm.n[0])) &&
                              coarse_kept(wavenumber(i1, dm.n[1]), dm.n[1]) && coarse_kept(i2, dm.n[2]);
            const KVec kv = kvec(dm, lin);
            double l = ipow(kv.k2, sp.p);
            if (l == 0.0) l = 1.0;
            const T f = (band_cut && !kept) ? T(0) : T(sign * pow(seg_alpha(sp, dm, lin) * l, expo));
            C2<T> g[3];
    #pragma unroll
            for (int c = 0; c < 3; ++c) g[c] = c < sp.dim ? gh.spec[c][lin] : cmk(T(0), T(0));
            if (sp.leray) leray_point(kv, sp.dim, g);
    #pragma unroll
            for (int c = 0; c < 3; ++c)
                if (c < sp.dim) sh.spec[c][lin] = cscale(g[c], f);
        }
    }
};

// Half spectra between a grid and the grid with half the cells per axis,
// on the coarse space; every other entry of the destination is zero.
// restrict: coarse(k) = scale fine(k);  prolong: fine(k) = scale coarse(k).

template <typename T>
struct SpecRestrictArgs {
    Dims df;
    Dims dc;
    SpecPtrs<T> fine;
    SpecPtrs<T> coarse;
    int count;
    T scale;
};
template <typename T>
struct SpecRestrictBody {
    static constexpr int kBlock = 256;
    using Args = SpecRestrictArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& df = args_.df;
        const Dims& dc = args_.dc;
        const SpecPtrs<T>& fine = args_.fine;
        const SpecPtrs<T>& coarse = args_.coarse;
        int count = args_.count;
        T scale = args_.scale;
        for (long long lin = bk.x * (long long)blockDim.x + threadIdx.x; lin < dc.NH;
             lin += (long long)bk.gx * blockDim.x) {
            const int i2 = (int)(lin % dc.n2h);
            const long long rest = lin / dc.n2h;
            const int i1 = (int)(rest % dc.n[1]), i0 = (int)(rest / dc.n[1]);
            const int k0 = dc.dim == 3 ? wavenumber(i0, dc.n[0]) : 0;
            const int k1 = wavenumber(i1, dc.n[1]);
            const bool keep = (dc.dim == 2 || coarse_kept(k0, dc.n[0])) && coarse_kept(k1, dc.n[1]) &&
                              coarse_kept(i2, dc.n[2]);
            long long src = 0;
            if (keep) {
                const int f0 = dc.dim == 3 ? (k0 < 0 ? k0 + df.n[0] : k0) : i0;
                const int f1 = k1 < 0 ? k1 + df.n[1] : k1;
                src = ((long long)f0 * df.n[1] + f1) * df.n2h + i2;
            }
            for (int c = 0; c < count; ++c)
                coarse.spec[c][lin] = keep ? cscale(fine.spec[c][src], scale) : cmk(T(0), T(0));
        }
    }
};

template <typename T>
struct SpecProlongArgs {
    Dims df;
    Dims dc;
    SpecPtrs<T> coarse;
    SpecPtrs<T> fine;
    int count;
    T scale;
};
template <typename T>
struct SpecProlongBody {
    static constexpr int kBlock = 256;
    using Args = SpecProlongArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& df = args_.df;
        const Dims& dc = args_.dc;
        const SpecPtrs<T>& coarse = args_.coarse;
        const SpecPtrs<T>& fine = args_.fine;
        int count = args_.count;
        T scale = args_.scale;
        for (long long lin = bk.x * (long long)blockDim.x + threadIdx.x; lin < df.NH;
             lin += (long long)bk.gx * blockDim.x) {
            const int i2 = (int)(lin % df.n2h);
            const long long rest = lin / df.n2h;
            const int i1 = (int)(rest % df.n[1]), i0 = (int)(rest / df.n[1]);
            const int k0 = df.dim == 3 ? wavenumber(i0, df.n[0]) : 0;
            const int k1 = wavenumber(i1, df.n[1]);
            const bool keep = (df.dim == 2 || coarse_kept(k0, dc.n[0])) && coarse_kept(k1, dc.n[1]) &&
                              coarse_kept(i2, dc.n[2]);
            long long src = 0;
            if (keep) {
                const int c0 = df.dim == 3 ? (k0 < 0 ? k0 + dc.n[0] : k0) : i0;
                const int c1 = k1 < 0 ? k1 + dc.n[1] : k1;
                src = ((long long)c0 * dc.n[1] + c1) * dc.n2h + i2;
            }
            for (int c = 0; c < count; ++c)
                fine.spec[c][lin] = keep ? cscale(coarse.spec[c][src], scale) : cmk(T(0), T(0));
        }
    }
};

// Cross terms of the regulariser along a line: with the half-spectrum
// weights (1 at k2 = 0 and at the Nyquist index, else 2),
//   res[0] = sum w l_p Re(vh conj(sh)),  res[1] = sum w l_p |sh|^2.
template <typename T>
struct SpecCrossArgs {
    Dims dm;
    SpecOpParams sp;
    SpecPtrs<double> vh;
    SpecPtrs<T> sh;
    double* partial;
};
template <typename T>
struct SpecCrossBody {
    static constexpr int kBlock = 256;
    using Args = SpecCrossArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const SpecOpParams& sp = args_.sp;
        const SpecPtrs<double>& vh = args_.vh;
        const SpecPtrs<T>& sh = args_.sh;
        double* partial = args_.partial;
        __shared__ double red[256 / 64];
        double a = 0.0, b = 0.0;
        const long long len = dm.NH / bk.gy, lo = bk.y * len;
        for (long long lin = lo + bk.x * (long long)blockDim.x + threadIdx.x; lin < lo + len;
             lin += (long long)bk.gx * blockDim.x) {
            const KVec kv = kvec(dm, lin);
            const int i2 = (int)(lin % dm.n2h);
            const double wl = ((i2 == 0 || 2 * i2 == dm.n[2]) ? 1.0 : 2.0) * ipow(kv.k2, sp.p);
    #pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c >= sp.dim) continue;
                const C2<double> z = vh.spec[c][lin];
                const C2<T> q = sh.spec[c][lin];
                a += wl * (z.x * double(q.x) + z.y * double(q.y));
                b += wl * (double(q.x) * double(q.x) + double(q.y) * double(q.y));
            }
        }
        const double ra = block_reduce<false>(a, red);
        const double rb = block_reduce<false>(b, red);
        if (threadIdx.x == 0) {
            partial[(long long)bk.y * bk.gx + bk.x] = ra;
            partial[(long long)(bk.gy + bk.y) * bk.gx + bk.x] = rb;
        }
    }
};

// vh[c] += rho * sh[c]  (FP64 spectrum of v updated along a line)
template <typename T>
struct SpecAxpyArgs {
    Dims dm;
    int dim;
    SpecPtrs<double> vh;
    SegCoef rc;
    SpecPtrs<T> sh;
};
template <typename T>
struct SpecAxpyBody {
    static constexpr int kBlock = 256;
    using Args = SpecAxpyArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        int dim = args_.dim;
        const SpecPtrs<double>& vh = args_.vh;
        const SegCoef& rc = args_.rc;
        const SpecPtrs<T>& sh = args_.sh;
        for (long long lin = bk.x * (long long)blockDim.x + threadIdx.x; lin < dm.NH;
             lin += (long long)bk.gx * blockDim.x) {
            const double rho = rc.c[spec_seg(dm, lin)];
    #pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c >= dim) continue;
                C2<double> z = vh.spec[c][lin];
                const C2<T> q = sh.spec[c][lin];
                z.x += rho * double(q.x);
                z.y += rho * double(q.y);
                vh.spec[c][lin] = z;
            }
        }
    }
};

template <typename T>
struct SpecRegvalueArgs {
    Dims dm;
    SpecOpParams sp;
    SpecPtrs<T> vh;
    double* partial;
};
template <typename T>
struct SpecRegvalueBody {
    static constexpr int kBlock = 256;
    using Args = SpecRegvalueArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const SpecOpParams& sp = args_.sp;
        const SpecPtrs<T>& vh = args_.vh;
        double* partial = args_.partial;
        __shared__ double sh[256 / 64];
        double acc = 0.0;
        const long long len = dm.NH / bk.gy, lo = bk.y * len;
        for (long long lin = lo + bk.x * (long long)blockDim.x + threadIdx.x; lin < lo + len;
             lin += (long long)bk.gx * blockDim.x) {
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
        if (threadIdx.x == 0) partial[(long long)bk.y * bk.gx + bk.x] = r;
    }
};

// blocks per stacked problem of a spectral reduction of nq quantities
inline int spec_red_blocks(const Dims& dm, int nq) {
    const int ns = spec_nseg(dm);
    int b = reduction_blocks(dm.NH / ns);
    const int cap = (64 * 1024) / (nq * ns);
    return b > cap ? (cap < 1 ? 1 : cap) : b;
}

inline int pointwise_blocks(long long n) {
    long long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

template <typename T>
hipError_t launch_deriv_axis(const Dims& dm, const SpectralPlans<T>& pl, int axis,
                             const T* const* F, const T* const* G, const double* w, int ntime,
                             int accumulate, T* out, hipStream_t st) {
    if (ntime < 1 || ntime > kMaxTime) return hipErrorInvalidValue;
    auto fill = [&](auto& a, int mt) {
        a.dm = dm;
        a.pl = pl.p[axis];
        a.axis = axis;
        a.pcshift = pc_shift_real(dm.n[axis], (int)sizeof(C2<T>), pencil_count(dm, axis, dm.n[2]),
                                  kDerivThreads);
        a.ntime = ntime;
        a.accumulate = accumulate;
        a.has_g = G != nullptr;
        a.out = out;
        for (int t = 0; t < mt; ++t) {
            a.F[t] = t < ntime ? F[t] : nullptr;
            a.G[t] = (G && t < ntime) ? G[t] : nullptr;
            a.w[t] = t < ntime ? w[t] : 0.0;
        }
    };
    const int L = dm.n[axis];
    const long long npen = pencil_count(dm, axis, dm.n[2]);
    const int PC = 1 << pc_shift_real(L, (int)sizeof(C2<T>), npen, kDerivThreads);
    const long long tiles = (npen + 2 * PC - 1) / (2 * PC);
    const size_t lds = fft_lds_bytes(PC, L, sizeof(C2<T>));
    if (ntime <= kGroupTime) {
        DerivArgs<T, kGroupTime> a;
        fill(a, kGroupTime);
        with_length(L, [&](auto lc) {
            constexpr int LCv = decltype(lc)::value;
            using Fam = MergeFamily<LCv, DerivAxisBody<T, LCv, kGroupTime>, DerivAxisAnyBody<T, kGroupTime>>;
            constexpr int PF = pc_shift_real_full(LCv > 0 ? LCv : 1, (int)sizeof(C2<T>), kDerivThreads);
            if constexpr (LCv > 0) {
                if (a.pcshift == PF) {
                    submit<DerivAxisBody<T, LCv, kGroupTime, PF>, Fam>(dim3((unsigned)tiles), lds, st, a);
                    return;
                }
            }
            submit<DerivAxisBody<T, LCv, kGroupTime>, Fam>(dim3((unsigned)tiles), lds, st, a);
        });
    } else {
        DerivArgs<T, kMaxTime> a;
        fill(a, kMaxTime);
        with_length(L, [&](auto lc) {
            constexpr int LCv = decltype(lc)::value;
            constexpr int PF = pc_shift_real_full(LCv > 0 ? LCv : 1, (int)sizeof(C2<T>), kDerivThreads);
            if constexpr (LCv > 0) {
                if (a.pcshift == PF) {
                    launch_now<DerivAxisBody<T, LCv, kMaxTime, PF>>(dim3((unsigned)tiles), lds, st, a);
                    return;
                }
            }
            launch_now<DerivAxisBody<T, LCv, kMaxTime>>(dim3((unsigned)tiles), lds, st, a);
        });
    }
    return hipGetLastError();
}

// A complex axis pass of compiled length LC (0: runtime plan) with NT = nt
// threads, compiled for the tile's pencil count when it is that of a large
// grid.
template <typename T, int LC>
void submit_c2c_axis(int nt, int sh, dim3 g, size_t lds, hipStream_t st, const C2cAxisArgs<T>& ca) {
    auto go = [&](auto ntc) {
        constexpr int NT = decltype(ntc)::value;
        using Fam = MergeFamily<LC, C2cAxisBody<T, LC, NT>, C2cAxisAnyBody<T, NT>>;
        constexpr int PF = pc_shift_cplx_full(LC > 0 ? LC : 1, (int)sizeof(C2<T>), NT);
        if constexpr (LC > 0) {
            if (sh == PF) {
                submit<C2cAxisBody<T, LC, NT, PF>, Fam>(g, lds, st, ca);
                return;
            }
        }
        submit<C2cAxisBody<T, LC, NT>, Fam>(g, lds, st, ca);
    };
    if (nt == kWideThreads)
        go(std::integral_constant<int, kWideThreads>{});
    else
        go(std::integral_constant<int, kFftThreads>{});
}
// The fused spectral pass, likewise.
template <typename T, int LC, int OP>
void submit_c2c_spec(int sh, dim3 g, size_t lds, hipStream_t st, const C2cSpecArgs<T>& ca) {
    using Fam = MergeFamily<LC, C2cSpecBody<T, LC, OP>, C2cSpecAnyBody<T, OP>>;
    constexpr int PF = pc_shift_cplx_full(LC > 0 ? LC : 1, (int)sizeof(C2<T>));
    if constexpr (LC > 0) {
        if (sh == PF) {
            submit<C2cSpecBody<T, LC, OP, PF>, Fam>(g, lds, st, ca);
            return;
        }
    }
    submit<C2cSpecBody<T, LC, OP>, Fam>(g, lds, st, ca);
}

template <typename TI, typename TC>
hipError_t launch_rfft(const Dims& dm, const SpectralPlans<TC>& pl, const TI* const* in,
                       C2<TC>* const* out, int count, hipStream_t st, int skip_last) {
    if (count < 1 || count > 3) return hipErrorInvalidValue;
    InPtrs<TI> ip{};
    SpecPtrs<TC> sp{};
    for (int c = 0; c < count; ++c) {
        ip.in[c] = in[c];
        sp.spec[c] = out[c];
    }
    {
        const int L = dm.n[2];
        const long long rows = (long long)dm.n[0] * dm.n[1];
        const int sh = pc_shift_real(L, (int)sizeof(C2<TC>), rows);
        const int PC = 1 << sh;
        dim3 g((unsigned)((rows + 2 * PC - 1) / (2 * PC)), count);
        const R2cRowsArgs<TI, TC> ra{dm, pl.p[2], sh, ip, sp};
        const size_t lds = fft_lds_bytes(PC, L, sizeof(C2<TC>));
        with_length(L, [&](auto lc) {
            constexpr int LC = decltype(lc)::value;
            using Fam = MergeFamily<LC, R2cRowsBody<TI, TC, LC>, R2cRowsAnyBody<TI, TC>>;
            constexpr int PF = pc_shift_real_full(LC > 0 ? LC : 1, (int)sizeof(C2<TC>), kFftThreads);
            if constexpr (LC > 0) {
                if (sh == PF) {
                    submit<R2cRowsBody<TI, TC, LC, PF>, Fam>(g, lds, st, ra);
                    return;
                }
            }
            submit<R2cRowsBody<TI, TC, LC>, Fam>(g, lds, st, ra);
        });
    }
    for (int axis = 1; axis >= 3 - dm.dim + (skip_last ? 1 : 0); --axis) {
        const int L = dm.n[axis];
        const long long npen = pencil_count(dm, axis, dm.n2h);
        const int nt = c2c_threads(L);
        const int sh = pc_shift_cplx(L, (int)sizeof(C2<TC>), npen, nt);
        const int PC = 1 << sh;
        dim3 g(strided_blocks((npen + PC - 1) / PC, kTilesPerBlock), count);
        const C2cAxisArgs<TC> ca{dm, pl.p[axis], axis, sh, -1, sp};
        const size_t lds = fft_lds_bytes(PC, L, sizeof(C2<TC>));
        with_length(L, [&](auto lc) { submit_c2c_axis<TC, decltype(lc)::value>(nt, sh, g, lds, st, ca); });
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_irfft(const Dims& dm, const SpectralPlans<T>& pl, C2<T>* const* spec,
                        T* const* out, const T* const* add, double scale, int count,
                        hipStream_t st, int skip_first) {
    if (count < 1 || count > 3) return hipErrorInvalidValue;
    SpecPtrs<T> sp{};
    OutPtrs<T> op{};
    for (int c = 0; c < count; ++c) {
        sp.spec[c] = spec[c];
        op.out[c] = out[c];
        op.add[c] = add ? add[c] : nullptr;
    }
    for (int axis = 3 - dm.dim + (skip_first ? 1 : 0); axis <= 1; ++axis) {
        const int L = dm.n[axis];
        const long long npen = pencil_count(dm, axis, dm.n2h);
        const int nt = c2c_threads(L);
        const int sh = pc_shift_cplx(L, (int)sizeof(C2<T>), npen, nt);
        const int PC = 1 << sh;
        dim3 g(strided_blocks((npen + PC - 1) / PC, kTilesPerBlock), count);
        const C2cAxisArgs<T> ca{dm, pl.p[axis], axis, sh, +1, sp};
        const size_t lds = fft_lds_bytes(PC, L, sizeof(C2<T>));
        with_length(L, [&](auto lc) { submit_c2c_axis<T, decltype(lc)::value>(nt, sh, g, lds, st, ca); });
    }
    {
        const int L = dm.n[2];
        const long long rows = (long long)dm.n[0] * dm.n[1];
        const int sh = pc_shift_real(L, (int)sizeof(C2<T>), rows);
        const int PC = 1 << sh;
        dim3 g((unsigned)((rows + 2 * PC - 1) / (2 * PC)), count);
        const C2rRowsArgs<T> ra{dm, pl.p[2], sh, T(scale), sp, op};
        const size_t lds = fft_lds_bytes(PC, L, sizeof(C2<T>));
        with_length(L, [&](auto lc) {
            constexpr int LC = decltype(lc)::value;
            using Fam = MergeFamily<LC, C2rRowsBody<T, LC>, C2rRowsAnyBody<T>>;
            constexpr int PF = pc_shift_real_full(LC > 0 ? LC : 1, (int)sizeof(C2<T>), kFftThreads);
            if constexpr (LC > 0) {
                if (sh == PF) {
                    submit<C2rRowsBody<T, LC, PF>, Fam>(g, lds, st, ra);
                    return;
                }
            }
            submit<C2rRowsBody<T, LC>, Fam>(g, lds, st, ra);
        });
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
    submit<SpecGradientBody<T>>(dim3(pointwise_blocks(dm.NH)), 0, st, SpecGradientArgs<T>{dm, sp, a, b, g});
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_precond(const Dims& dm, const SpecOpParams& sp, C2<T>* const* gh,
                               C2<T>* const* sh, C2<T>* const* keep, hipStream_t st) {
    SpecPtrs<T> a{}, b{}, k{};
    for (int c = 0; c < sp.dim; ++c) {
        a.spec[c] = gh[c];
        b.spec[c] = sh[c];
        k.spec[c] = keep ? keep[c] : nullptr;
    }
    submit<SpecPrecondBody<T>>(dim3(pointwise_blocks(dm.NH)), 0, st, SpecPrecondArgs<T>{dm, sp, a, b, k, keep != nullptr});
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_fused(const Dims& dm, const SpectralPlans<T>& pl, int op,
                             const SpecOpParams& sp, C2<T>* const* io, C2<double>* const* vh,
                             C2<T>* const* keep, hipStream_t st, C2<T>* const* pre) {
    if (sp.dim != dm.dim || (op != kSpecGrad && op != kSpecPrecond)) return hipErrorInvalidValue;
    if (op == kSpecGrad && (keep == nullptr) != (pre == nullptr)) return hipErrorInvalidValue;
    SpecPtrs<T> a{}, k{}, pr{};
    SpecPtrs<double> v{};
    for (int c = 0; c < sp.dim; ++c) {
        a.spec[c] = io[c];
        k.spec[c] = keep ? keep[c] : nullptr;
        v.spec[c] = vh ? vh[c] : nullptr;
        pr.spec[c] = pre ? pre[c] : nullptr;
    }
    if (op == kSpecGrad && !vh) return hipErrorInvalidValue;
    const int axis = 3 - dm.dim;
    const int L = dm.n[axis];
    const long long npen = pencil_count(dm, axis, dm.n2h);
    const int sh = pc_shift_cplx(L, (int)sizeof(C2<T>), npen);
    const int PC = 1 << sh;
    // one tile per workgroup: a tile carries every component, so the grid is a
    // third of that of a single-field pass and needs all its workgroups
    const unsigned g = strided_blocks((npen + PC - 1) / PC, 1);
    const C2cSpecArgs<T> ca{dm, pl.p[axis], axis, sh, sp, a, v, k, keep != nullptr, pr};
    const size_t lds = fft_lds_bytes(PC, L, sizeof(C2<T>));
    with_length(L, [&](auto lc) {
        if (op == kSpecGrad)
            submit_c2c_spec<T, decltype(lc)::value, kSpecGrad>(sh, dim3(g), lds, st, ca);
        else
            submit_c2c_spec<T, decltype(lc)::value, kSpecPrecond>(sh, dim3(g), lds, st, ca);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_pow(const Dims& dm, const SpecOpParams& sp, C2<T>* const* gh,
                           C2<T>* const* sh, double expo, double sign, int band_cut,
                           hipStream_t st) {
    SpecPtrs<T> a{}, b{};
    for (int c = 0; c < sp.dim; ++c) {
        a.spec[c] = gh[c];
        b.spec[c] = sh[c];
    }
    submit<SpecPowBody<T>>(dim3(pointwise_blocks(dm.NH)), 0, st, SpecPowArgs<T>{dm, sp, a, b, expo, sign, band_cut});
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_resample(const Dims& df, const Dims& dc, C2<T>* const* src,
                                C2<T>* const* dst, int count, int to_coarse, double scale,
                                hipStream_t st) {
    if (count < 1 || count > 3 || df.dim != dc.dim) return hipErrorInvalidValue;
    for (int a = 3 - df.dim; a < 3; ++a)
        if (df.n[a] != 2 * dc.n[a]) return hipErrorInvalidValue;
    if (df.dim == 2 && df.n[0] != dc.n[0]) return hipErrorInvalidValue;
    SpecPtrs<T> s{}, d{};
    for (int c = 0; c < count; ++c) {
        s.spec[c] = src[c];
        d.spec[c] = dst[c];
    }
    if (to_coarse)
        submit<SpecRestrictBody<T>>(dim3(pointwise_blocks(dc.NH)), 0, st, SpecRestrictArgs<T>{df, dc, s, d, count, T(scale)});
    else
        submit<SpecProlongBody<T>>(dim3(pointwise_blocks(df.NH)), 0, st, SpecProlongArgs<T>{df, dc, s, d, count, T(scale)});
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_cross(const Dims& dm, const SpecOpParams& sp, C2<double>* const* vh,
                             C2<T>* const* sh, double* partial, double* res, hipStream_t st) {
    SpecPtrs<double> a{};
    SpecPtrs<T> b{};
    for (int c = 0; c < sp.dim; ++c) {
        a.spec[c] = vh[c];
        b.spec[c] = sh[c];
    }
    const int ns = spec_nseg(dm), nb = spec_red_blocks(dm, 2);
    submit<SpecCrossBody<T>>(dim3(nb, ns), 0, st, SpecCrossArgs<T>{dm, sp, a, b, partial});
    launch_finish<false>(partial, nb, 2 * ns, res, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_axpy(const Dims& dm, int dim, C2<double>* const* vh, const double* rho,
                            C2<T>* const* sh, hipStream_t st) {
    SpecPtrs<double> a{};
    SpecPtrs<T> b{};
    for (int c = 0; c < dim; ++c) {
        a.spec[c] = vh[c];
        b.spec[c] = sh[c];
    }
    const int ns = spec_nseg(dm);
    if (ns > kMaxSeg) return hipErrorInvalidValue;
    SegCoef rc{};
    for (int i = 0; i < ns; ++i) rc.c[i] = rho[i];
    submit<SpecAxpyBody<T>>(dim3(pointwise_blocks(dm.NH)), 0, st, SpecAxpyArgs<T>{dm, dim, a, rc, b});
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spec_regvalue(const Dims& dm, const SpecOpParams& sp, C2<T>* const* vh,
                                double* partial, double* res, hipStream_t st) {
    SpecPtrs<T> a{};
    for (int c = 0; c < sp.dim; ++c) a.spec[c] = vh[c];
    const int ns = spec_nseg(dm), nb = spec_red_blocks(dm, 1);
    submit<SpecRegvalueBody<T>>(dim3(nb, ns), 0, st, SpecRegvalueArgs<T>{dm, sp, a, partial});
    launch_finish<false>(partial, nb, ns, res, st);
    return hipGetLastError();
}

#define GAN_INST(T)                                                                               \
    template hipError_t launch_deriv_axis<T>(const Dims&, const SpectralPlans<T>&, int,           \
                                             const T* const*, const T* const*, const double*,     \
                                             int, int, T*, hipStream_t);                          \
    template hipError_t launch_rfft<T, T>(const Dims&, const SpectralPlans<T>&, const T* const*,  \
                                          C2<T>* const*, int, hipStream_t, int);                  \
    template hipError_t launch_irfft<T>(const Dims&, const SpectralPlans<T>&, C2<T>* const*,      \
                                        T* const*, const T* const*, double, int, hipStream_t,     \
                                        int);                                                     \
    template hipError_t launch_spec_fused<T>(const Dims&, const SpectralPlans<T>&, int,           \
                                             const SpecOpParams&, C2<T>* const*,                  \
                                             C2<double>* const*, C2<T>* const*, hipStream_t,      \
                                             C2<T>* const*);                                      \
    template hipError_t launch_spec_gradient<T>(const Dims&, const SpecOpParams&,                 \
                                                C2<double>* const*, C2<T>* const*, C2<T>* const*, \
                                                hipStream_t);                                     \
    template hipError_t launch_spec_precond<T>(const Dims&, const SpecOpParams&, C2<T>* const*,   \
                                               C2<T>* const*, C2<T>* const*, hipStream_t);        \
    template hipError_t launch_spec_cross<T>(const Dims&, const SpecOpParams&, C2<double>* const*, \
                                             C2<T>* const*, double*, double*, hipStream_t);       \
    template hipError_t launch_spec_axpy<T>(const Dims&, int, C2<double>* const*, const double*,  \
                                            C2<T>* const*, hipStream_t);                          \
    template hipError_t launch_spec_regvalue<T>(const Dims&, const SpecOpParams&, C2<T>* const*,  \
                                                double*, double*, hipStream_t);                   \
    template hipError_t launch_spec_pow<T>(const Dims&, const SpecOpParams&, C2<T>* const*,       \
                                           C2<T>* const*, double, double, int, hipStream_t);      \
    template hipError_t launch_spec_resample<T>(const Dims&, const Dims&, C2<T>* const*,          \
                                                C2<T>* const*, int, int, double, hipStream_t);
GAN_INST(float)
GAN_INST(double)
#undef GAN_INST
template hipError_t launch_rfft<float, double>(const Dims&, const SpectralPlans<double>&,
                                               const float* const*, C2<double>* const*, int,
                                               hipStream_t, int);

}  // namespace gan
