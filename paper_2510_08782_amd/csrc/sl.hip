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
// 2-D: 64 x 32).  Before the gather it reduces, over the tile, the smallest
// and largest floor of the departure displacement along every axis, and
// stages the source region those departure points can touch: along each
// axis the tile shifted by the smallest floor, widened by the spread of the
// floors plus the 3 extra nodes of the cubic stencil.  The region's capacity
// is fixed per variant (spread up to S cells per axis); every tap then comes
// from LDS at a compile-time offset from one base address per point.  Only
// the spread of the displacements within a tile must fit, not their size, so
// long but smooth displacements (large line-search trials) stay on the LDS
// path.  A tile whose spread exceeds S reads its taps directly from global
// memory instead.  Both paths give the same values: only where the taps are
// read from changes.
#include <cmath>

#include "launch.hpp"
#include "group.hpp"
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

// The 4 x taps of one row, weighted.  When the stencil does not wrap the taps
// are consecutive elements and move with one 16-byte load per 4 bytes of
// element width (global loads need only element alignment on this target);
// wrapped stencils read them one by one.
template <typename T>
struct Quad {
    T v[4];
};
template <typename T>
__device__ inline T row_taps(const T* __restrict__ row, const int* o, bool contig, const T* w) {
    if (contig) {
        Quad<T> q;
        __builtin_memcpy(&q, row + o[0], sizeof(q));
        return w[0] * q.v[0] + w[1] * q.v[1] + w[2] * q.v[2] + w[3] * q.v[3];
    }
    return w[0] * row[o[0]] + w[1] * row[o[1]] + w[2] * row[o[2]] + w[3] * row[o[3]];
}

// Direct (L1/L2) gather of one field at point (i0,i1,i2) + (d0,d1,d2).  Used
// by tiles whose departure points spread too far for the staged window, e.g.
// the first line-search trials from v = 0, so it is written for scattered
// access: 16 row loads per point instead of 64 element loads.
template <typename T, int DIM>
__device__ inline T gather_global(const Dims& dm, const T* __restrict__ s, int i0, int i1, int i2,
                                  T d0, T d1, T d2) {
    int o1[4], o2[4];
    T w1[4], w2[4];
    axis_taps(i1, d1, dm.n[1], dm.n[2], o1, w1);
    axis_taps(i2, d2, dm.n[2], 1, o2, w2);
    const bool contig = o2[3] == o2[0] + 3;
    T acc = T(0);
    if constexpr (DIM == 3) {
        int o0[4];
        T w0[4];
        axis_taps(i0, d0, dm.n[0], dm.n[1] * dm.n[2], o0, w0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            T sa = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) sa += w1[b] * row_taps(s + o0[a] + o1[b], o2, contig, w2);
            acc += w0[a] * sa;
        }
    } else {
        // 2-D: axis 0 indexes independent slices
        const T* sl = s + (long long)i0 * dm.n[1] * dm.n[2];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc += w1[b] * row_taps(sl + o1[b], o2, contig, w2);
    }
    return acc;
}

// ---- tile geometry -----------------------------------------------------------
// 3-D: threads (32 x 8), each owns P = TZ points along z.  2-D: threads
// (64 x 4), each owns P points along y (tile 64 x 4P; P = 8, 4 or 2, the
// variant chosen per grid size by the tile autotuner, see Dims::tile).  S is
// the capacity of the staged region: up to S cells of spread of the
// displacement floors per axis.
#ifndef GAN_PX3
#define GAN_PX3 48  // LDS row pitch of the 3-D windows (words)
#endif
#ifndef GAN_TZ_F32
#define GAN_TZ_F32 2  // points per thread along z of the 3-D FP32 tiles
#endif
template <typename T_, int DIM_, int S_,
          int P_ = (DIM_ == 3 ? (sizeof(T_) == 4 ? GAN_TZ_F32 : 4) : kTile2Default)>
struct Tile;
template <typename T_, int S_, int TZ_>
struct Tile<T_, 3, S_, TZ_> {
    using T = T_;
    static constexpr int DIM = 3;
    static constexpr int TX = 32, TY = 8, TZ = TZ_;
    static constexpr int S = S_;
    static constexpr int RX = TX + S + 3, RY = TY + S + 3, RZ = TZ + S + 3;
    // LDS row pitch: the two rows a wavefront reads (lanes 0-31 and 32-63)
    // start half the banks apart
    static constexpr int PX = GAN_PX3;
    static constexpr int PZ = PX * RY;  // plane pitch
    static_assert(RX + 2 <= PX && PX % 2 == 0, "row pitch: even, and room for the pair past a row");
    static constexpr int PTS = TZ;  // points per thread
    static constexpr int LDSN = PZ * RZ + 2;  // elements per staged field (even)
};
template <typename T_, int S_, int P_>
struct Tile<T_, 2, S_, P_> {
    using T = T_;
    static constexpr int DIM = 2;
    static constexpr int TX = 64, TY = 4 * P_, TZ = 1;
    static constexpr int S = S_;
    static constexpr int RX = TX + S + 3, RY = TY + S + 3, RZ = 1;
    static constexpr int PX = (RX + 1) & ~1;  // a wavefront reads one row; even pitch
    static constexpr int PZ = PX * RY;
    static constexpr int PTS = P_;
    static constexpr int LDSN = PZ * RZ + 2;
};

// LDS bytes of one staged field.  Rows start at even element offsets and the
// region ends with two spare elements, so that the FP32 interpolation can read
// every row as aligned pairs (the last pair may reach one element past a row).
template <class C>
constexpr size_t tile_lds_bytes() {
    return sizeof(typename C::T) * C::LDSN;
}

// g mod n in [0, n): the common in-range case costs one compare.
__device__ inline int wrapn(int g, int n) {
    return (static_cast<unsigned>(g) < static_cast<unsigned>(n)) ? g : pmod(g, n);
}

// The staged region of a tile: along axis a (0: x, 1: y, 2: z) it starts at
// tile origin + lo[a] - 1 and spans ext[a] = T_a + spread_a + 3 nodes.
struct Window {
    int lo[3];
    int ext[3];
    bool lds;  // every spread fits the variant's capacity
};

__device__ inline int wave_min_i(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
    return x;
}
__device__ inline int wave_max_i(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
    return x;
}

// Floor of a displacement as used for the window; the taps of the LDS path
// use the unclamped floor, which agrees whenever the window is taken (all
// floors of the tile within +-2^20).
template <typename T>
__device__ inline int disp_floor(T d) {
    return static_cast<int>(floor(clamp_disp(d)));
}

// The window of a tile whose displacement floors span [m[a], M[a]] per axis
// (x, y, z order).
template <class C>
__device__ inline Window window_from(const int (&m_)[3], const int (&M_)[3]) {
    Window w;
    const int T3[3] = {C::TX, C::TY, C::TZ};
    w.lds = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int m = m_[a], M = M_[a];
        if (a == 2 && C::DIM == 2) m = M = 0;  // slice axis: no interpolation
        const int spread = M - m;
        w.lds = w.lds && spread <= C::S && m >= -(1 << 20) && M <= (1 << 20);
        w.lo[a] = m;
        w.ext[a] = (a == 2 && C::DIM == 2) ? 1 : T3[a] + spread + 3;
    }
    return w;
}

// Block-wide window from per-thread floor ranges fmn/fmx (x, y, z order).
// red: 6 ints per wave of LDS.  Contains a barrier.
template <class C>
__device__ inline Window tile_window(const int (&fmn)[3], const int (&fmx)[3], int* red,
                                     int* entry = nullptr) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int m = wave_min_i(fmn[a]);
        const int M = wave_max_i(fmx[a]);
        if (lane == 0) {
            red[wave * 6 + a] = m;
            red[wave * 6 + 3 + a] = M;
        }
    }
    __syncthreads();
    int m[3], M[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m[a] = red[a];
        M[a] = red[3 + a];
#pragma unroll
        for (int q = 1; q < kThreads / 64; ++q) {
            m[a] = min(m[a], red[q * 6 + a]);
            M[a] = max(M[a], red[q * 6 + 3 + a]);
        }
        // the same in every lane: keep it in scalar registers
        m[a] = __builtin_amdgcn_readfirstlane(m[a]);
        M[a] = __builtin_amdgcn_readfirstlane(M[a]);
    }
    if (entry && threadIdx.x < 6) {
        const int i = threadIdx.x;
        entry[i] = i == 0 ? m[0] : i == 1 ? m[1] : i == 2 ? m[2] : i == 3 ? M[0] : i == 4 ? M[1] : M[2];
    }
    return window_from<C>(m, M);
}

// g mod n for a wave-uniform g: the window origins lie within one period of
// the grid in all but extreme displacements, so the common cases are scalar
// compares and the division only runs for the rest.
__device__ inline int wrap_uniform(int g, int n) {
    if (g >= 0 && g < n) return g;
    if (g < 0 && g >= -n) return g + n;
    if (g >= n && g < 2 * n) return g - n;
    return pmod(g, n);
}

// Stage src over the window of the tile with origin (x0, y0, z0).
// Global-to-LDS loads (global_load_lds_dword): a wavefront walks the rows of
// the region and moves each row with one instruction per 64 dwords, lane l
// writing dword l of the row; the wrapped x index of every lane is computed
// once.  The wave's rows are described in parallel, one row per lane (its
// global offset and its LDS offset), and the issue loop only reads them back
// from the lanes, so that it carries no division, wrap or branch per row.
// The descriptions avoid integer division too: the row's plane comes from a
// float reciprocal of the row count per plane (exact for these small
// integers), and the grid rows wrap by comparison from the wrapped window
// origin.  All of a wave's row loads are in flight together and no VGPRs
// hold the data.  FP64 rows move as pairs of dwords.  The LDS layout keeps
// the variant's row pitch PX and plane pitch PZ.  Ends with a barrier unless
// WAIT is false.
template <class C, bool WAIT = true>
__device__ inline void stage(const Dims& dm, const typename C::T* __restrict__ src,
                             typename C::T* lds, int x0, int y0, int z0, const Window& w) {
    using T = typename C::T;
    constexpr int W = sizeof(T) / 4;                  // dwords per element
    constexpr int NW = kThreads / 64;
    constexpr int XP = (W * C::RX + 63) / 64;         // dword passes per row
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n0 = dm.n[0], n1 = dm.n[1], n2 = dm.n[2];
    const int ex = w.ext[0], ey = w.ext[1], rows = w.ext[1] * w.ext[2];
    const int ox = wrap_uniform(x0 + w.lo[0] - 1, n2);
    const int oy = wrap_uniform(y0 + w.lo[1] - 1, n1);
    // 2-D: axis 0 indexes independent slices (no interpolation across it)
    const int oz = C::DIM == 3 ? wrap_uniform(z0 + w.lo[2] - 1, n0) : z0;
    int goff[XP];                                    // dword offset of the lane's element in a row
    bool xin[XP];
#pragma unroll
    for (int u = 0; u < XP; ++u) {
        const int d = lane + 64 * u;
        xin[u] = d < W * ex;
        int gx = ox + d / W;
        while (gx >= n2) gx -= n2;
        goff[u] = W * gx + d % W;
    }
    // (r + 1/2) / ey is at least 1 / (2 ey) away from an integer; for the
    // row counts here (r < 2^21) the float error of the product is smaller
    const float rey = 1.0f / static_cast<float>(ey);
    // this wave's rows are r = wave + NW i, i < cnt
    const int cnt = rows > wave ? (rows - wave + NW - 1) / NW : 0;
    for (int i0 = 0; i0 < cnt; i0 += 64) {
        const int r = wave + NW * (i0 + lane);
        const int rz = static_cast<int>((static_cast<float>(r) + 0.5f) * rey);
        const int ry = r - rz * ey;
        int gy = oy + ry;
        while (gy >= n1) gy -= n1;
        int gz = z0;
        if constexpr (C::DIM == 3) {
            gz = oz + rz;
            while (gz >= n0) gz -= n0;
        }
        const int grow = (gz * n1 + gy) * n2;  // elements; N < 2^31
        const int lrow = rz * C::PZ + ry * C::PX;
        const int m = min(64, cnt - i0);
        // The row descriptions are read back from the lanes (readlane, wave
        // uniform) before the loads are masked to the lanes inside the row:
        // reading a lane's value under a mask that excludes it would read a
        // register that lane never wrote.
        int j = 0;
        for (; j + 4 <= m; j += 4) {
            int go[4], lo[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                go[q] = __builtin_amdgcn_readlane(grow, j + q);
                lo[q] = __builtin_amdgcn_readlane(lrow, j + q);
            }
#pragma unroll
            for (int u = 0; u < XP; ++u)
                if (xin[u]) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        __builtin_amdgcn_global_load_lds(
                            reinterpret_cast<const unsigned*>(src + go[q]) + goff[u],
                            reinterpret_cast<unsigned*>(lds + lo[q]) + 64 * u, 4, 0, 0);
                }
        }
        for (; j < m; ++j) {
            const int go = __builtin_amdgcn_readlane(grow, j);
            const int lo = __builtin_amdgcn_readlane(lrow, j);
#pragma unroll
            for (int u = 0; u < XP; ++u)
                if (xin[u])
                    __builtin_amdgcn_global_load_lds(reinterpret_cast<const unsigned*>(src + go) + goff[u],
                                                     reinterpret_cast<unsigned*>(lds + lo) + 64 * u, 4, 0,
                                                     0);
        }
    }
    if constexpr (WAIT) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

// Tap base and weights along one axis for the LDS path: local index of the
// node f-1 for point index li within the tile, the window starting at
// floor minimum lo (minus one).
// The window (from the tile's floor ranges) always contains the stencil; the
// clamp only keeps the LDS address inside the region if a window table were
// stale.  Built with GAN_CHECK_TAPS, a stencil outside the staged extent ext
// instead poisons its weights with NaN, so that the evaluation fails with
// GANMRES_ENONFINITE rather than returning silently wrong values.
template <typename T, int R>
__device__ inline int lds_axis(int li, T disp, int lo, int ext, T* w) {
    const T fl = floor(disp);
    lagrange4(disp - fl, w);
    int l = li + static_cast<int>(fl) - lo;
#ifdef GAN_CHECK_TAPS
    if (l < 0 || l > ext - 4) w[0] = w[1] = w[2] = w[3] = T(NAN);
#else
    (void)ext;
#endif
    l = l < 0 ? 0 : (l > R - 4 ? R - 4 : l);
    return l;
}

// Stencil of one departure point in the staged window: offset of its first
// tap and the cubic weights per axis.
template <typename T>
struct Stencil {
    int base;
    T wx[4], wy[4], wz[4];
};

template <class C>
__device__ inline Stencil<typename C::T> lds_stencil(const Window& win, int lx, int ly, int lz,
                                                     typename C::T d0, typename C::T d1,
                                                     typename C::T d2) {
    using T = typename C::T;
    Stencil<T> st;
    const int bx = lds_axis<T, C::RX>(lx, d2, win.lo[0], win.ext[0], st.wx);
    const int by = lds_axis<T, C::RY>(ly, d1, win.lo[1], win.ext[1], st.wy);
    if constexpr (C::DIM == 3) {
        const int bz = lds_axis<T, C::RZ>(lz, d0, win.lo[2], win.ext[2], st.wz);
        st.base = bz * C::PZ + by * C::PX + bx;
    } else {
        st.base = by * C::PX + bx;
    }
    return st;
}

// Offset of plane a of a stencil plus d, held in a register of its own: the
// row reads of the plane then address it with the instruction's immediate
// offset (rows up to 3 PX + 3 elements away), where otherwise each read of a
// plane beyond the first would get an address addition of its own.
template <class C>
__device__ inline int plane_offset(int base, int a, int d = 0) {
    int o = base + a * C::PZ + d;
    if (a > 0 || d != 0) asm("" : "+v"(o));
    return o;
}

// One 8-byte LDS read.  The reads are volatile so that the compiler keeps them
// as separate ds_read_b64: merged into ds_read2_b64 they move data at about
// two thirds of the rate on this target.
template <typename T>
struct Pair {
    T x, y;
};
__device__ inline Pair<float> lds_pair(const float* p) {
    typedef float V2 __attribute__((ext_vector_type(2)));
    typedef const volatile __attribute__((address_space(3))) V2 LV2;
    const V2 v = *(LV2*)(p);
    return Pair<float>{v.x, v.y};
}
// One LDS element, kept as a read of its own in the same way.
template <typename T>
__device__ inline T lds_one(const T* p) {
    typedef const volatile __attribute__((address_space(3))) T LT;
    return *(LT*)(p);
}

// Tensor-product cubic interpolation of a staged field at a stencil.
//
// FP32: the four x taps of a row start at any element, but LDS reads of 8
// bytes are fast only when aligned (a misaligned one is serialised, and two
// 4-byte reads take half again as long as one aligned 8-byte read).  Each row
// is therefore read as aligned pairs starting at the even element at or
// below the first tap, and the row is contracted with five x weights: the
// four cubic weights, shifted by one when the first tap is odd.  The fifth
// element is read on its own (4 bytes): the one after the four taps' pairs
// when the first tap is odd, a repeat of the third when it is even (its
// weight is then zero), so that no element outside the staged row enters the
// sum.
//
// FP64: every tap is one aligned 8-byte read; they are kept as separate
// reads too, which take less time than the paired form.
template <class C>
__device__ inline typename C::T lds_interp(const typename C::T* lds,
                                           const Stencil<typename C::T>& st) {
    using T = typename C::T;
    if constexpr (sizeof(T) == 4) {
        const bool odd = st.base & 1;
        const int e = st.base & ~1;
        const T u0 = odd ? T(0) : st.wx[0], u1 = odd ? st.wx[0] : st.wx[1];
        const T u2 = odd ? st.wx[1] : st.wx[2], u3 = odd ? st.wx[2] : st.wx[3];
        const T u4 = odd ? st.wx[3] : T(0);
        const int d3 = odd ? 4 : 2;
        const int nplanes = C::DIM == 3 ? 4 : 1;
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < nplanes; ++a) {
            const T* plane = lds + plane_offset<C>(e, a);
            const T* third = lds + plane_offset<C>(e, a, d3);
            Pair<T> q[4][2];
            T t[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                q[b][0] = lds_pair(plane + b * C::PX);
                q[b][1] = lds_pair(plane + b * C::PX + 2);
                t[b] = lds_one(third + b * C::PX);
            }
            T sa = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                sa += st.wy[b] * (u0 * q[b][0].x + u1 * q[b][0].y + u2 * q[b][1].x +
                                  u3 * q[b][1].y + u4 * t[b]);
            acc = C::DIM == 3 ? acc + st.wz[a] * sa : sa;
        }
        return acc;
    } else {
        const T* base = lds + st.base;
        T acc = T(0);
        if constexpr (C::DIM == 3) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                T sa = T(0);
                const T* plane = lds + plane_offset<C>(st.base, a);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const T* row = plane + b * C::PX;
                    sa += st.wy[b] * (st.wx[0] * lds_one(row) + st.wx[1] * lds_one(row + 1) +
                                      st.wx[2] * lds_one(row + 2) + st.wx[3] * lds_one(row + 3));
                }
                acc += st.wz[a] * sa;
            }
        } else {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const T* row = base + b * C::PX;
                acc += st.wy[b] * (st.wx[0] * lds_one(row) + st.wx[1] * lds_one(row + 1) +
                                   st.wx[2] * lds_one(row + 2) + st.wx[3] * lds_one(row + 3));
            }
        }
        return acc;
    }
}

// Interpolate from the staged window at tile-local point (lx,ly,lz) displaced by d.
template <class C>
__device__ inline typename C::T gather_lds(const typename C::T* lds, const Window& win, int lx,
                                           int ly, int lz, typename C::T d0, typename C::T d1,
                                           typename C::T d2) {
    return lds_interp<C>(lds, lds_stencil<C>(win, lx, ly, lz, d0, d1, d2));
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b mod 8), each with its own L2.  Tiles are numbered x-fastest, then y,
// then z, and XCD k is given the contiguous range of tiles
// [k ceil(T/8), (k+1) ceil(T/8)): a slab whose halos are mostly read from
// the same L2 instead of once per XCD.
constexpr int kXcds = 8;
constexpr int kWinInts = 8;  // ints per tile in a window table

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
    int x0, y0, z0, t;
    bool valid;
    __device__ PointMap(const Dims& dm, const Blk& bk) {
        const int ntx = (dm.n[2] + C::TX - 1) / C::TX;
        const int nty = (dm.n[1] + C::TY - 1) / C::TY;
        const int T = tile_count<C>(dm);
        const int per = (T + kXcds - 1) / kXcds;
        t = (bk.x % kXcds) * per + bk.x / kXcds;
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
// r = I[src] at the point; EPI 0: out = r;  1: out = fac r;  3: out = fac + r;
// 2 (source factor, src = delta): out = 1 + sgn h/2 (r + delta) + h^2/2 delta r
template <typename T, int EPI>
__device__ inline T step_epilogue(T r, const T* __restrict__ src, const T* __restrict__ fac,
                                  long long lin, T ht, T sgn) {
    if constexpr (EPI == 1) r *= fac[lin];
    if constexpr (EPI == 3) r += fac[lin];
    if constexpr (EPI == 2) {
        const T dc = src[lin];
        r = T(1) + sgn * T(0.5) * ht * (r + dc) + T(0.5) * ht * ht * dc * r;
    }
    return r;
}

// LDS = true: tiles whose window fits (the others return at once);
// LDS = false: the remaining tiles, every tap read from global memory.  Two
// kernels, so that the LDS path does not carry the direct gather's registers;
// the second is launched only when the spread bound allows a tile to
// exceed the window.
//
// table (nullable): the window table of disp.  With table_write = 0 it holds
// every tile's floor ranges, the window is known at once, and the staging of
// the source is in flight while the displacements load.  With table_write = 1
// (the first gather over a new field) the LDS kernel reduces its windows as
// without a table and records them there.
template <typename T>
struct SlStepArgs {
    Dims dm;
    const T* src;
    const T* disp;
    const T* fac;
    T ht;
    T sgn;
    T* out;
    int* table;
    int table_write;
};
template <class C, int EPI, bool LDS>
struct SlStepBody {
    static constexpr int kBlock = kThreads;
    using Args = SlStepArgs<typename C::T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const typename C::T* __restrict__ src = args_.src;
        const typename C::T* __restrict__ disp = args_.disp;
        const typename C::T* __restrict__ fac = args_.fac;
        typename C::T ht = args_.ht;
        typename C::T sgn = args_.sgn;
        typename C::T* __restrict__ out = args_.out;
        int* __restrict__ table = args_.table;
        int table_write = args_.table_write;
        using T = typename C::T;
        constexpr int DIM = C::DIM;
        extern __shared__ double2 sl_smem[];
        T* lds = reinterpret_cast<T*>(sl_smem);
        __shared__ int red[6 * (kThreads / 64)];
        const PointMap<C> pm(dm, bk);
        if (!pm.valid) return;
        Window win{};
        const bool use_table = table && !table_write;
        if (use_table) {
            const int* e = table + (long long)pm.t * kWinInts;
            const int m[3] = {e[0], e[1], e[2]}, M[3] = {e[3], e[4], e[5]};
            win = window_from<C>(m, M);
            if (win.lds != LDS) return;
            if constexpr (LDS) stage<C, false>(dm, src, lds, pm.x0, pm.y0, pm.z0, win);
        }
        const long long N = dm.N;
        // displacements of the thread's points and their floor ranges
        T d0[C::PTS], d1[C::PTS], d2[C::PTS];
        long long lin[C::PTS];
        bool in[C::PTS];
        int fmn[3] = {1 << 30, 1 << 30, 1 << 30}, fmx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    #pragma unroll
        for (int k = 0; k < C::PTS; ++k) {
            int lx, ly, lz;
            pm.local(k, lx, ly, lz);
            const int i2 = pm.x0 + lx, i1 = pm.y0 + ly, i0 = pm.z0 + lz;
            in[k] = i2 < dm.n[2] && i1 < dm.n[1] && i0 < dm.n[0];
            lin[k] = ((long long)i0 * dm.n[1] + i1) * dm.n[2] + i2;
            // every lane loads (a point outside the grid reads element 0), so
            // that the loads of all points are in flight together
            const long long lc = in[k] ? lin[k] : 0;
            if constexpr (DIM == 3) {
                d0[k] = disp[lc];
                d1[k] = disp[N + lc];
                d2[k] = disp[2 * N + lc];
            } else {
                d0[k] = T(0);
                d1[k] = disp[lc];
                d2[k] = disp[N + lc];
            }
        }
        if (!use_table) {
    #pragma unroll
            for (int k = 0; k < C::PTS; ++k) {
                const int f[3] = {disp_floor(d2[k]), disp_floor(d1[k]), disp_floor(d0[k])};
    #pragma unroll
                for (int q = 0; q < 3; ++q) {
                    fmn[q] = in[k] ? min(fmn[q], f[q]) : fmn[q];
                    fmx[q] = in[k] ? max(fmx[q], f[q]) : fmx[q];
                }
            }
        }
        if (!use_table) {
            win = tile_window<C>(fmn, fmx, red,
                                 (LDS && table) ? table + (long long)pm.t * kWinInts : nullptr);
            if (win.lds != LDS) return;
            if constexpr (LDS) stage<C>(dm, src, lds, pm.x0, pm.y0, pm.z0, win);
        } else if constexpr (LDS) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
    #pragma unroll
        for (int k = 0; k < C::PTS; ++k) {
            if (!in[k]) continue;
            int lx, ly, lz;
            pm.local(k, lx, ly, lz);
            T r;
            if constexpr (LDS)
                r = gather_lds<C>(lds, win, lx, ly, lz, d0[k], d1[k], d2[k]);
            else
                r = gather_global<T, DIM>(dm, src, pm.z0 + lz, pm.y0 + ly, pm.x0 + lx, d0[k], d1[k],
                                          d2[k]);
            out[lin[k]] = step_epilogue<T, EPI>(r, src, fac, lin[k], ht, sgn);
        }
    }
};

// ---- characteristics -------------------------------------------------------------
// dX = -(u + I[u](i - u)) / 2 (state, +v) and dY = (u + I[u](i + u)) / 2
// (adjoint, -v), u_c = s_c v_c.  The predictor points only depend on u at the
// grid point, so the window is known before any staging; component c of v is
// then staged in LDS in turn.  With both directions the window covers both
// sets of predictor points.
template <typename T>
struct CharacteristicsArgs {
    Dims dm;
    const T* v;
    T s0;
    T s1;
    T s2;
    T* dX;
    T* dY;
};
template <class C, bool DOX, bool DOY, bool LDS>
struct CharacteristicsBody {
    static constexpr int kBlock = kThreads;
    using Args = CharacteristicsArgs<typename C::T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const typename C::T* __restrict__ v = args_.v;
        typename C::T s0 = args_.s0;
        typename C::T s1 = args_.s1;
        typename C::T s2 = args_.s2;
        typename C::T* __restrict__ dX = args_.dX;
        typename C::T* __restrict__ dY = args_.dY;
        using T = typename C::T;
        constexpr int DIM = C::DIM;
        extern __shared__ double2 sl_smem[];
        T* lds = reinterpret_cast<T*>(sl_smem);
        __shared__ int red[6 * (kThreads / 64)];
        const PointMap<C> pm(dm, bk);
        if (!pm.valid) return;
        const long long N = dm.N;
        const T s[3] = {s0, s1, s2};
        // u at the thread's points, all loads in flight together (a point
        // outside the grid reads element 0 and is masked)
        T u[C::PTS][DIM];
        bool inp[C::PTS];
    #pragma unroll
        for (int k = 0; k < C::PTS; ++k) {
            int lx, ly, lz;
            pm.local(k, lx, ly, lz);
            const int i2 = pm.x0 + lx, i1 = pm.y0 + ly, i0 = pm.z0 + lz;
            inp[k] = i2 < dm.n[2] && i1 < dm.n[1] && i0 < dm.n[0];
            const long long lc = inp[k] ? ((long long)i0 * dm.n[1] + i1) * dm.n[2] + i2 : 0;
    #pragma unroll
            for (int c = 0; c < DIM; ++c) u[k][c] = v[c * N + lc];
        }
        int fmn[3] = {1 << 30, 1 << 30, 1 << 30}, fmx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    #pragma unroll
        for (int k = 0; k < C::PTS; ++k) {
    #pragma unroll
            for (int c = 0; c < DIM; ++c) {
                u[k][c] = inp[k] ? u[k][c] * s[c] : T(0);
                const int q = DIM - 1 - c;  // axis slot: x, y, z
                if (DOX) {
                    const int f = disp_floor(-u[k][c]);
                    fmn[q] = inp[k] ? min(fmn[q], f) : fmn[q];
                    fmx[q] = inp[k] ? max(fmx[q], f) : fmx[q];
                }
                if (DOY) {
                    const int f = disp_floor(u[k][c]);
                    fmn[q] = inp[k] ? min(fmn[q], f) : fmn[q];
                    fmx[q] = inp[k] ? max(fmx[q], f) : fmx[q];
                }
            }
        }
        const Window win = tile_window<C>(fmn, fmx, red);
        if (win.lds != LDS) return;
        // the stencils of the predictor points (weights, first tap) serve every
        // component: computed once, before the first staging
        Stencil<T> stx[C::PTS], sty[C::PTS];
        if constexpr (LDS) {
    #pragma unroll
            for (int k = 0; k < C::PTS; ++k) {
                int lx, ly, lz;
                pm.local(k, lx, ly, lz);
                const T e0 = DIM == 3 ? u[k][0] : T(0), e1 = DIM == 3 ? u[k][1] : u[k][0];
                const T e2 = DIM == 3 ? u[k][2] : u[k][1];
                if (DOX) stx[k] = lds_stencil<C>(win, lx, ly, lz, -e0, -e1, -e2);
                if (DOY) sty[k] = lds_stencil<C>(win, lx, ly, lz, e0, e1, e2);
            }
        }
    #pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const T* vc = v + c * N;
            if constexpr (LDS) {
                if (c > 0) __syncthreads();
                stage<C>(dm, vc, lds, pm.x0, pm.y0, pm.z0, win);
            }
    #pragma unroll
            for (int k = 0; k < C::PTS; ++k) {
                if (!inp[k]) continue;
                int lx, ly, lz;
                pm.local(k, lx, ly, lz);
                const int i2 = pm.x0 + lx, i1 = pm.y0 + ly, i0 = pm.z0 + lz;
                const long long lin = ((long long)i0 * dm.n[1] + i1) * dm.n[2] + i2;
                const T e0 = DIM == 3 ? u[k][0] : T(0), e1 = DIM == 3 ? u[k][1] : u[k][0];
                const T e2 = DIM == 3 ? u[k][2] : u[k][1];
                if (DOX) {
                    const T iv = LDS ? lds_interp<C>(lds, stx[k])
                                     : gather_global<T, DIM>(dm, vc, i0, i1, i2, -e0, -e1, -e2);
                    dX[c * N + lin] = T(-0.5) * (u[k][c] + s[c] * iv);
                }
                if (DOY) {
                    const T iv = LDS ? lds_interp<C>(lds, sty[k])
                                     : gather_global<T, DIM>(dm, vc, i0, i1, i2, e0, e1, e2);
                    dY[c * N + lin] = T(0.5) * (u[k][c] + s[c] * iv);
                }
            }
        }
    }
};

// Characteristics with every component of v staged at once (DIM windows in
// LDS): the stencil of a predictor point (weights, first tap) is computed
// once and serves all DIM components, and with both directions one staging
// serves X and Y.  Tiles that do not fit are left to
// characteristics_kernel<C, DOX, DOY, false>.
template <typename T>
struct CharacteristicsAllArgs {
    Dims dm;
    const T* v;
    T s0;
    T s1;
    T s2;
    T* dX;
    T* dY;
};
template <class C, bool DOX, bool DOY>
struct CharacteristicsAllBody {
    static constexpr int kBlock = kThreads;
    using Args = CharacteristicsAllArgs<typename C::T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const Dims& dm = args_.dm;
        const typename C::T* __restrict__ v = args_.v;
        typename C::T s0 = args_.s0;
        typename C::T s1 = args_.s1;
        typename C::T s2 = args_.s2;
        typename C::T* __restrict__ dX = args_.dX;
        typename C::T* __restrict__ dY = args_.dY;
        using T = typename C::T;
        constexpr int DIM = C::DIM;
        constexpr int PLANE = C::LDSN;  // elements per staged component
        extern __shared__ double2 sl_smem[];
        T* lds = reinterpret_cast<T*>(sl_smem);
        __shared__ int red[6 * (kThreads / 64)];
        const PointMap<C> pm(dm, bk);
        if (!pm.valid) return;
        const long long N = dm.N;
        const T s[3] = {s0, s1, s2};
        int fmn[3] = {1 << 30, 1 << 30, 1 << 30}, fmx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
        // every lane loads (a point outside the grid reads element 0), so that
        // the loads of all points are in flight together
        T ev[C::PTS][DIM];
        bool inp[C::PTS];
    #pragma unroll
        for (int k = 0; k < C::PTS; ++k) {
            int lx, ly, lz;
            pm.local(k, lx, ly, lz);
            const int i2 = pm.x0 + lx, i1 = pm.y0 + ly, i0 = pm.z0 + lz;
            inp[k] = i2 < dm.n[2] && i1 < dm.n[1] && i0 < dm.n[0];
            const long long lc = inp[k] ? ((long long)i0 * dm.n[1] + i1) * dm.n[2] + i2 : 0;
    #pragma unroll
            for (int c = 0; c < DIM; ++c) ev[k][c] = v[c * N + lc];
        }
    #pragma unroll
        for (int k = 0; k < C::PTS; ++k) {
    #pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const T e = ev[k][c] * s[c];
                const int q = DIM - 1 - c;  // axis slot: x, y, z
                if (DOX) {
                    const int f = disp_floor(-e);
                    fmn[q] = inp[k] ? min(fmn[q], f) : fmn[q];
                    fmx[q] = inp[k] ? max(fmx[q], f) : fmx[q];
                }
                if (DOY) {
                    const int f = disp_floor(e);
                    fmn[q] = inp[k] ? min(fmn[q], f) : fmn[q];
                    fmx[q] = inp[k] ? max(fmx[q], f) : fmx[q];
                }
            }
        }
        const Window win = tile_window<C>(fmn, fmx, red);
        if (!win.lds) return;
    #pragma unroll
        for (int c = 0; c < DIM; ++c) {
            if (c + 1 < DIM)
                stage<C, false>(dm, v + c * N, lds + c * PLANE, pm.x0, pm.y0, pm.z0, win);
            else
                stage<C, true>(dm, v + c * N, lds + c * PLANE, pm.x0, pm.y0, pm.z0, win);
        }
    #pragma unroll
        for (int k = 0; k < C::PTS; ++k) {
            if (!inp[k]) continue;
            int lx, ly, lz;
            pm.local(k, lx, ly, lz);
            const long long lin =
                ((long long)(pm.z0 + lz) * dm.n[1] + (pm.y0 + ly)) * dm.n[2] + (pm.x0 + lx);
            T u[DIM];
    #pragma unroll
            for (int c = 0; c < DIM; ++c) u[c] = ev[k][c] * s[c];
            const T e0 = DIM == 3 ? u[0] : T(0), e1 = DIM == 3 ? u[1] : u[0];
            const T e2 = DIM == 3 ? u[2] : u[1];
            if (DOX) {
                const Stencil<T> st = lds_stencil<C>(win, lx, ly, lz, -e0, -e1, -e2);
    #pragma unroll
                for (int c = 0; c < DIM; ++c)
                    dX[c * N + lin] = T(-0.5) * (u[c] + s[c] * lds_interp<C>(lds + c * PLANE, st));
            }
            if (DOY) {
                const Stencil<T> st = lds_stencil<C>(win, lx, ly, lz, e0, e1, e2);
    #pragma unroll
                for (int c = 0; c < DIM; ++c)
                    dY[c * N + lin] = T(0.5) * (u[c] + s[c] * lds_interp<C>(lds + c * PLANE, st));
            }
        }
    }
};

// max_c max_i |s_c v_c(i)| (NaN/inf counted as 1e30): FP64 block partials
template <typename T>
struct VelocityMaxArgs {
    const T* v;
    long long N;
    int dim;
    double s0;
    double s1;
    double s2;
    int vec;
    double* partial;
};
template <typename T>
struct VelocityMaxBody {
    static constexpr int kBlock = kThreads;
    using Args = VelocityMaxArgs<T>;
    __device__ __forceinline__ static void run(const Args& args_, const Blk& bk) {
        const T* __restrict__ v = args_.v;
        long long N = args_.N;
        int dim = args_.dim;
        double s0 = args_.s0;
        double s1 = args_.s1;
        double s2 = args_.s2;
        int vec = args_.vec;
        double* __restrict__ partial = args_.partial;
        __shared__ double sh[kThreads / 64];
        const double s[3] = {s0, s1, s2};
        double m = 0.0;
        bool bad = false;
        constexpr int W = 16 / (int)sizeof(T);
        struct alignas(16) V {
            T x[W];
        };
        for (int c = 0; c < dim; ++c) {
            // max |v_c| in the field's type, scaled once (s_c > 0); with vec every
            // thread moves 16 bytes at a time
            T mc = T(0);
            if (vec) {
                const V* row = reinterpret_cast<const V*>(v + c * N);
                for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < N / W;
                     i += (long long)bk.gx * blockDim.x) {
                    const V q = row[i];
    #pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const T a = fabs(q.x[w]);
                        bad = bad || !(a == a);
                        mc = fmax(mc, a);
                    }
                }
            } else {
                for (long long i = bk.x * (long long)blockDim.x + threadIdx.x; i < N;
                     i += (long long)bk.gx * blockDim.x) {
                    const T a = fabs(v[c * N + i]);
                    bad = bad || !(a == a);
                    mc = fmax(mc, a);
                }
            }
            m = fmax(m, double(mc) * s[c]);
        }
        if (bad || !(m <= 1.0e30)) m = 1.0e30;
        const double r = block_reduce<true>(m, sh);
        if (threadIdx.x == 0) partial[bk.x] = r;
    }
};

// Variant choice from a bound on the spread of the displacement floors over
// the field (cells; a displacement bound B gives floor(B) + ceil(B), which is
// odd unless B is an integer): the smallest capacity that covers it; beyond
// the largest, the largest runs and only tiles whose own spread exceeds it
// gather from global memory.  FP32 3-D: 2, 3 or 8 (a bound of 4 would need B
// to be exactly 2); FP64 3-D: 2, 3 or 4, the largest that fits the LDS.
template <typename T, int DIM>
int pick_capacity(int spread) {
    if (DIM == 2) return spread <= 8 ? 8 : 16;
    if (sizeof(T) == 8) return spread <= 2 ? 2 : (spread <= 3 ? 3 : 4);
    return spread <= 2 ? 2 : (spread <= 3 ? 3 : 8);
}

// Bodies of merged 2-D launches: classes of a group handle may run different
// tile variants (Dims::tile); the variant of each class is dispatched here.
template <typename F>
__device__ __forceinline__ void with_tile_dev(int tile, F&& f) {
    switch (tile) {
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        default: f(std::integral_constant<int, 8>{}); break;
    }
}
template <typename T, int S, int EPI, bool LDS>
struct SlStepAnyBody {
    static constexpr int kBlock = kThreads;
    using Args = SlStepArgs<T>;
    __device__ __forceinline__ static void run(const Args& a, const Blk& bk) {
        with_tile_dev(a.dm.tile, [&](auto p) __attribute__((always_inline)) {
            SlStepBody<Tile<T, 2, S, decltype(p)::value>, EPI, LDS>::run(a, bk);
        });
    }
};
template <typename T, int S, bool DOX, bool DOY, bool LDS>
struct CharacteristicsAnyBody {
    static constexpr int kBlock = kThreads;
    using Args = CharacteristicsArgs<T>;
    __device__ __forceinline__ static void run(const Args& a, const Blk& bk) {
        with_tile_dev(a.dm.tile, [&](auto p) __attribute__((always_inline)) {
            CharacteristicsBody<Tile<T, 2, S, decltype(p)::value>, DOX, DOY, LDS>::run(a, bk);
        });
    }
};
template <typename T, int S, bool DOX, bool DOY>
struct CharacteristicsAllAnyBody {
    static constexpr int kBlock = kThreads;
    using Args = CharacteristicsAllArgs<T>;
    __device__ __forceinline__ static void run(const Args& a, const Blk& bk) {
        with_tile_dev(a.dm.tile, [&](auto p) __attribute__((always_inline)) {
            CharacteristicsAllBody<Tile<T, 2, S, decltype(p)::value>, DOX, DOY>::run(a, bk);
        });
    }
};
// The merged family of a tile: its variant-dispatching body in 2-D, the
// tile's own body in 3-D (one variant per capacity).
template <class C, class Body, class AnyBody>
using TileFamily = typename std::conditional<C::DIM == 2, AnyBody, Body>::type;

template <class C, bool DOX, bool DOY, bool LDS>
void char_submit(const Dims& dm, size_t lds, hipStream_t st, const CharacteristicsArgs<typename C::T>& a) {
    using B = CharacteristicsBody<C, DOX, DOY, LDS>;
    submit<B, TileFamily<C, B, CharacteristicsAnyBody<typename C::T, C::S, DOX, DOY, LDS>>>(
        dim3(tile_blocks<C>(dm)), lds, st, a);
}

template <class C, bool DOX, bool DOY>
void char_launch(const Dims& dm, const typename C::T* v, const double* s, int spread,
                 typename C::T* dX, typename C::T* dY, hipStream_t st) {
    using T = typename C::T;
    const CharacteristicsArgs<T> a{dm, v, T(s[0]), T(s[1]), T(C::DIM == 3 ? s[2] : 0.0), dX, dY};
    char_submit<C, DOX, DOY, true>(dm, tile_lds_bytes<C>(), st, a);
    if (spread > C::S) char_submit<C, DOX, DOY, false>(dm, 0, st, a);
}

template <class C, bool DOX, bool DOY>
void char_all_launch(const Dims& dm, const typename C::T* v, const double* s, int spread,
                     typename C::T* dX, typename C::T* dY, hipStream_t st) {
    using T = typename C::T;
    using B = CharacteristicsAllBody<C, DOX, DOY>;
    const CharacteristicsAllArgs<T> a{dm, v, T(s[0]), T(s[1]), T(C::DIM == 3 ? s[2] : 0.0), dX, dY};
    submit<B, TileFamily<C, B, CharacteristicsAllAnyBody<T, C::S, DOX, DOY>>>(
        dim3(tile_blocks<C>(dm)), C::DIM * tile_lds_bytes<C>(), st, a);
    if (spread > C::S)
        char_submit<C, DOX, DOY, false>(dm, 0, st,
                                        CharacteristicsArgs<T>{dm, v, a.s0, a.s1, a.s2, dX, dY});
}

// LDS per workgroup on gfx950
constexpr size_t kMaxLds = 160 * 1024;

template <class C>
void char_dirs(const Dims& dm, const typename C::T* v, const double* s, int spread,
               typename C::T* dX, typename C::T* dY, hipStream_t st) {
    using T = typename C::T;
    // both directions: all components staged at once (one staging and one
    // stencil per point serve X and Y), on the gather's tiles, where the d
    // windows take at most half the LDS: in 2-D, and in 3-D FP32 with
    // capacities 2 and 3 (2 planes per tile, three workgroups per CU).  3-D
    // FP64 (4 planes per tile) and capacity 8 never fit and stage one
    // component at a time, as a single direction always does (that keeps
    // more workgroups per CU)
    using CA = C;
    if constexpr (C::DIM * tile_lds_bytes<CA>() <= kMaxLds / 2) {
        if (dX && dY) {
            char_all_launch<CA, true, true>(dm, v, s, spread, dX, dY, st);
            return;
        }
    }
    // one component staged at a time, one launch per direction in 3-D
    if (C::DIM == 3 || !(dX && dY)) {
        if (dX) char_launch<C, true, false>(dm, v, s, spread, dX, dY, st);
        if (dY) char_launch<C, false, true>(dm, v, s, spread, dX, dY, st);
    } else {
        char_launch<C, true, true>(dm, v, s, spread, dX, dY, st);
    }
}

template <class C, int EPI>
void step_kernels(const Dims& dm, const typename C::T* src, const typename C::T* disp,
                  const typename C::T* fac, double ht, double sgn, int spread,
                  typename C::T* out, int* table, int table_write, hipStream_t st) {
    using T = typename C::T;
    using BL = SlStepBody<C, EPI, true>;
    using BG = SlStepBody<C, EPI, false>;
    submit<BL, TileFamily<C, BL, SlStepAnyBody<T, C::S, EPI, true>>>(
        dim3(tile_blocks<C>(dm)), tile_lds_bytes<C>(), st,
        SlStepArgs<T>{dm, src, disp, fac, T(ht), T(sgn), out, table, table_write});
    // the direct-gather kernel reads the table only once it is complete
    if (spread > C::S)
        submit<BG, TileFamily<C, BG, SlStepAnyBody<T, C::S, EPI, false>>>(
            dim3(tile_blocks<C>(dm)), 0, st,
            SlStepArgs<T>{dm, src, disp, fac, T(ht), T(sgn), out, table, 0});
}

template <class C>
void step_launch(const Dims& dm, const typename C::T* src, const typename C::T* disp,
                 const typename C::T* fac, int spread, typename C::T* out, int* table,
                 int tw, hipStream_t st) {
    if (fac) step_kernels<C, 1>(dm, src, disp, fac, 0.0, 0.0, spread, out, table, tw, st);
    else step_kernels<C, 0>(dm, src, disp, fac, 0.0, 0.0, spread, out, table, tw, st);
}

template <class C>
void add_launch(const Dims& dm, const typename C::T* src, const typename C::T* disp,
                const typename C::T* add, int spread, typename C::T* out, int* table, int tw,
                hipStream_t st) {
    step_kernels<C, 3>(dm, src, disp, add, 0.0, 0.0, spread, out, table, tw, st);
}

template <class C>
void factor_launch(const Dims& dm, const typename C::T* delta, const typename C::T* disp,
                   double ht, double sgn, int spread, typename C::T* out, int* table, int tw,
                   hipStream_t st) {
    step_kernels<C, 2>(dm, delta, disp, nullptr, ht, sgn, spread, out, table, tw, st);
}

// Calls f(Tile<...>{}) with the variant chosen for `spread`.
template <typename T, typename F>
void dispatch_tile(const Dims& dm, int spread, F&& f) {
    if (dm.dim == 3) {
        const int c = pick_capacity<T, 3>(spread);
        if (c == 2) f(Tile<T, 3, 2>{});
        else if (c == 3) f(Tile<T, 3, 3>{});
        else if constexpr (sizeof(T) == 8) f(Tile<T, 3, 4>{});
        else f(Tile<T, 3, 8>{});
    } else {
        // the 2-D tile variant (points per thread) chosen for this grid size
        auto cap = [&](auto p) {
            constexpr int P = decltype(p)::value;
            if (pick_capacity<T, 2>(spread) == 8) f(Tile<T, 2, 8, P>{});
            else f(Tile<T, 2, 16, P>{});
        };
        if (dm.tile == 2) cap(std::integral_constant<int, 2>{});
        else if (dm.tile == 4) cap(std::integral_constant<int, 4>{});
        else cap(std::integral_constant<int, kTile2Default>{});
    }
}

}  // namespace

int spread_bound(double B) {
    if (!(B <= 1.0e6)) return 1 << 21;
    return static_cast<int>(std::floor(B) + std::ceil(B));
}

int displacement_bound(double umax, int dim) {
    // |X| = |u(i) + I[u](xi*)| / 2 <= (1 + 1.25^d) max|u| / 2: the cubic
    // Lagrange weights have absolute sum at most 1.25 per axis
    if (!(umax <= 1.0e6)) return 1 << 21;
    return spread_bound(0.5 * (1.0 + std::pow(1.25, dim)) * umax * (1.0 + 1e-6));
}

template <typename T>
hipError_t launch_velocity_max(const Dims& dm, const T* v, const double* s, double* partial,
                               double* res, hipStream_t st) {
    const int nb = reduction_blocks(dm.N);
    constexpr int W = 16 / (int)sizeof(T);
    const int vec = (dm.N % W == 0 && (reinterpret_cast<unsigned long long>(v) & 15) == 0) ? 1 : 0;
    submit<VelocityMaxBody<T>>(dim3(nb), 0, st, VelocityMaxArgs<T>{v, dm.N, dm.dim, s[0], s[1],
                                                    dm.dim == 3 ? s[2] : 0.0, vec, partial});
    launch_finish<true>(partial, nb, 1, res, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_characteristics(const Dims& dm, const T* v, const double* s, int spread, T* dX,
                                  T* dY, hipStream_t st) {
    dispatch_tile<T>(dm, spread, [&](auto tile) {
        char_dirs<decltype(tile)>(dm, v, s, spread, dX, dY, st);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sl_step(const Dims& dm, const T* src, const T* disp, const T* fac, int spread,
                          T* out, hipStream_t st, int* table, int table_write) {
    dispatch_tile<T>(dm, spread, [&](auto tile) {
        step_launch<decltype(tile)>(dm, src, disp, fac, spread, out, table, table_write, st);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sl_step_add(const Dims& dm, const T* src, const T* disp, const T* add,
                              int spread, T* out, hipStream_t st, int* table, int table_write) {
    dispatch_tile<T>(dm, spread, [&](auto tile) {
        add_launch<decltype(tile)>(dm, src, disp, add, spread, out, table, table_write, st);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_source_factor(const Dims& dm, const T* delta, const T* disp, double ht,
                                double sgn, int spread, T* out, hipStream_t st, int* table,
                                int table_write) {
    dispatch_tile<T>(dm, spread, [&](auto tile) {
        factor_launch<decltype(tile)>(dm, delta, disp, ht, sgn, spread, out, table, table_write, st);
    });
    return hipGetLastError();
}

// The tile geometry does not depend on the window capacity: one table serves
// every capacity.  In 2-D it is sized for the smallest tile variant (the most
// tiles), so that any variant the autotuner picks fits.
template <typename T>
long long window_table_ints(const Dims& dm0) {
    Dims dm = dm0;
    if (dm.dim == 2) dm.tile = 2;
    long long n = 0;
    dispatch_tile<T>(dm, 0, [&](auto tile) {
        using C = decltype(tile);
        n = (long long)tile_count<C>(dm) * kWinInts;
    });
    return n;
}



#define GAN_INST(T)                                                                               \
    template hipError_t launch_velocity_max<T>(const Dims&, const T*, const double*, double*,     \
                                               double*, hipStream_t);                             \
    template hipError_t launch_characteristics<T>(const Dims&, const T*, const double*, int, T*,  \
                                                  T*, hipStream_t);                               \
    template hipError_t launch_sl_step<T>(const Dims&, const T*, const T*, const T*, int, T*,     \
                                          hipStream_t, int*, int);                                \
    template hipError_t launch_sl_step_add<T>(const Dims&, const T*, const T*, const T*, int, T*, \
                                              hipStream_t, int*, int);                            \
    template hipError_t launch_source_factor<T>(const Dims&, const T*, const T*, double, double,  \
                                                int, T*, hipStream_t, int*, int);                 \
    template long long window_table_ints<T>(const Dims&);
GAN_INST(float)
GAN_INST(double)
#undef GAN_INST

}  // namespace gan
