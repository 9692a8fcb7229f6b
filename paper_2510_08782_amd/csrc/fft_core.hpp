// Mixed-radix (8/4/2/3) Stockham autosort FFT on data resident in LDS.
//
// Layout: PC pencils of length L interleaved as buf[lpad(i * PC + p)], so
// that the threads of a wavefront that share a butterfly index j touch
// consecutive words.  One pass of radix R turns the L/R length-R sub-transforms of the
// current stage into sub-transforms of length Ns*R:
//   inputs  a_r = in[j + r L/R]                      (r = 0..R-1)
//   twiddle a_r *= W^(k r L/(Ns R)),  k = j mod Ns,  W = exp(dir 2 pi i / L)
//   a R-point DFT with sign dir, then
//   outputs out[(j / Ns) Ns R + k + r Ns]
// which leaves the result in natural order after the last pass.
// dir = -1: forward (unnormalised), dir = +1: inverse (unnormalised).
#pragma once

#include "common.hpp"

namespace gan {

// LDS slot of complex element c of a transform buffer: one pad element after
// every 16.  Accesses that stride over the pencil-interleaved layout (the
// transposes between row-major global data and the tile, the first Stockham
// pass) then spread over the LDS banks instead of hitting one bank per
// stride.  A buffer of n elements occupies lpad_size(n) slots.
__host__ __device__ inline int lpad(int c) { return c + (c >> 4); }
__host__ __device__ inline int lpad_size(int n) { return n + (n >> 4) + 1; }

template <typename T, int R>
__host__ __device__ inline void dft_small(C2<T>* a, int dir) {
    const T s = static_cast<T>(dir);
    if constexpr (R == 2) {
        C2<T> t0 = a[0];
        a[0] = cadd(t0, a[1]);
        a[1] = csub(t0, a[1]);
    } else if constexpr (R == 3) {
        const T c3 = static_cast<T>(0.86602540378443864676);  // sqrt(3)/2
        C2<T> t1 = cadd(a[1], a[2]);
        C2<T> t2 = csub(a[0], cscale(t1, static_cast<T>(0.5)));
        C2<T> t3 = cmuli(csub(a[1], a[2]), s * c3);
        a[0] = cadd(a[0], t1);
        a[1] = cadd(t2, t3);
        a[2] = csub(t2, t3);
    } else if constexpr (R == 4) {
        C2<T> s02 = cadd(a[0], a[2]);
        C2<T> d02 = csub(a[0], a[2]);
        C2<T> s13 = cadd(a[1], a[3]);
        C2<T> d13 = cmuli(csub(a[1], a[3]), s);  // dir * i * (a1 - a3)
        a[0] = cadd(s02, s13);
        a[2] = csub(s02, s13);
        a[1] = cadd(d02, d13);
        a[3] = csub(d02, d13);
    } else if constexpr (R == 8) {
        // two radix-4 DFTs on even and odd samples, then a radix-2 merge
        const T h = static_cast<T>(0.70710678118654752440);
        C2<T> e[4] = {a[0], a[2], a[4], a[6]};
        C2<T> o[4] = {a[1], a[3], a[5], a[7]};
        dft_small<T, 4>(e, dir);
        dft_small<T, 4>(o, dir);
        // twiddles exp(dir 2 pi i q / 8), q = 0..3
        C2<T> o1 = cmk(h * (o[1].x - s * o[1].y), h * (o[1].y + s * o[1].x));
        C2<T> o2 = cmuli(o[2], s);
        C2<T> o3 = cmk(h * (-o[3].x - s * o[3].y), h * (-o[3].y + s * o[3].x));
        a[0] = cadd(e[0], o[0]);
        a[4] = csub(e[0], o[0]);
        a[1] = cadd(e[1], o1);
        a[5] = csub(e[1], o1);
        a[2] = cadd(e[2], o2);
        a[6] = csub(e[2], o2);
        a[3] = cadd(e[3], o3);
        a[7] = csub(e[3], o3);
    }
}

// One butterfly (index t in [0, PC * L / R)) of a Stockham pass.
template <typename T, int R>
__host__ __device__ inline void stockham_butterfly(const C2<T>* in, C2<T>* out, int t, int L,
                                                   int pcshift, int Ns, const C2<T>* tw, int dir) {
    const int PC = 1 << pcshift;
    const int p = t & (PC - 1);
    const int j = t >> pcshift;
    const int nb = L / R;
    const int k = j % Ns;
    C2<T> a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = in[lpad(((j + r * nb) << pcshift) + p)];
    if (Ns > 1) {
        const int step = L / (Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C2<T> w = tw[k * r * step];
            if (dir > 0) w.y = -w.y;
            a[r] = cmul(a[r], w);
        }
    }
    dft_small<T, R>(a, dir);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[lpad(((base + r * Ns) << pcshift) + p)] = a[r];
}

template <typename T>
__host__ __device__ inline void stockham_dispatch(int R, const C2<T>* in, C2<T>* out, int t, int L,
                                                  int pcshift, int Ns, const C2<T>* tw, int dir) {
    switch (R) {
        case 8: stockham_butterfly<T, 8>(in, out, t, L, pcshift, Ns, tw, dir); break;
        case 4: stockham_butterfly<T, 4>(in, out, t, L, pcshift, Ns, tw, dir); break;
        case 3: stockham_butterfly<T, 3>(in, out, t, L, pcshift, Ns, tw, dir); break;
        default: stockham_butterfly<T, 2>(in, out, t, L, pcshift, Ns, tw, dir); break;
    }
}

// Radix plan of make_radices below as a compile-time value.
struct RadixPlanCT {
    int n;
    int r[16];
};
constexpr RadixPlanCT radix_plan_ct(int L) {
    RadixPlanCT P{0, {}};
    int m = L, p2 = 0, p3 = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++p2;
    }
    while (m % 3 == 0) {
        m /= 3;
        ++p3;
    }
    while (p2 >= 3) {
        P.r[P.n++] = 8;
        p2 -= 3;
    }
    if (p2 == 2) P.r[P.n++] = 4;
    if (p2 == 1) P.r[P.n++] = 2;
    for (int i = 0; i < p3; ++i) P.r[P.n++] = 3;
    return P;
}

// Stockham butterfly with the transform length L and the stage's sub-length
// NS known at compile time: every division and modulus by them is constant.
// DERIV (last stage of a forward transform only): each output, at its final
// position i of the pencil, is multiplied by i k_i / L before it is stored
// (k_i the wavenumber with the Nyquist entry zero), so that a derivative needs
// no pass of its own over the spectrum.
// PCS >= 0: the tile's log2 pencil count is this constant (pcshift is then
// ignored).  lpad(c + 16 m) = lpad(c) + 17 m, so where the element stride
// between the R inputs (outputs) of a butterfly, in slots of the interleaved
// tile, is a multiple of 16, their LDS slots are one base plus constant
// offsets: one address per butterfly instead of one per element.
template <typename T, int R, int L, int NS, bool DERIV = false, int PCS = -1>
__device__ inline void stockham_butterfly_ct(const C2<T>* in, C2<T>* out, int t, int pcshift,
                                             const C2<T>* tw, int dir, T inv_l = T(0)) {
    if constexpr (PCS >= 0) {
        constexpr int PC = 1 << PCS;
        constexpr int nb = L / R;
        const int p = t & (PC - 1);
        const int j = t >> PCS;
        const int k = j % NS;
        C2<T> a[R];
        if constexpr ((nb * PC) % 16 == 0) {
            const C2<T>* src = in + lpad(j * PC + p);
    #pragma unroll
            for (int r = 0; r < R; ++r) a[r] = src[r * (nb * PC / 16 * 17)];
        } else {
    #pragma unroll
            for (int r = 0; r < R; ++r) a[r] = in[lpad((j + r * nb) * PC + p)];
        }
        if constexpr (NS > 1) {
            constexpr int step = L / (NS * R);
            const int ks = k * step;
    #pragma unroll
            for (int r = 1; r < R; ++r) {
                C2<T> w = tw[r * ks];
                if (dir > 0) w.y = -w.y;
                a[r] = cmul(a[r], w);
            }
        }
        dft_small<T, R>(a, dir);
        const int base = (j / NS) * NS * R + k;
        if constexpr (DERIV) {
    #pragma unroll
            for (int r = 0; r < R; ++r) a[r] = cmuli(a[r], T(wavenumber_odd(base + r * NS, L)) * inv_l);
        }
        if constexpr ((NS * PC) % 16 == 0) {
            C2<T>* dst = out + lpad(base * PC + p);
    #pragma unroll
            for (int r = 0; r < R; ++r) dst[r * (NS * PC / 16 * 17)] = a[r];
        } else {
    #pragma unroll
            for (int r = 0; r < R; ++r) out[lpad((base + r * NS) * PC + p)] = a[r];
        }
        return;
    }
    const int PC = 1 << pcshift;
    const int p = t & (PC - 1);
    const int j = t >> pcshift;
    constexpr int nb = L / R;
    const int k = j % NS;
    C2<T> a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = in[lpad(((j + r * nb) << pcshift) + p)];
    if constexpr (NS > 1) {
        constexpr int step = L / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C2<T> w = tw[k * r * step];
            if (dir > 0) w.y = -w.y;
            a[r] = cmul(a[r], w);
        }
    }
    dft_small<T, R>(a, dir);
    const int base = (j / NS) * NS * R + k;
    if constexpr (DERIV) {
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = cmuli(a[r], T(wavenumber_odd(base + r * NS, L)) * inv_l);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) out[lpad(((base + r * NS) << pcshift) + p)] = a[r];
}

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)
// block_fft for a compile-time length L (NT threads per block): the radix
// sequence, the stage lengths and the twiddle strides are constants.
// DERIV: the last stage applies the derivative factor (see
// stockham_butterfly_ct; forward transforms, dir = -1).
// PCS >= 0: the log2 pencil count of the tile as a constant (see
// stockham_butterfly_ct).
template <typename T, int L, int NT, int S = 0, int NS = 1, bool DERIV = false, int PCS = -1>
__device__ inline C2<T>* block_fft_ct(C2<T>* a, C2<T>* b, const C2<T>* tw, int pcshift, int dir,
                                      T inv_l = T(0)) {
    constexpr RadixPlanCT P = radix_plan_ct(L);
    if constexpr (S == P.n) {
        return a;
    } else {
        constexpr int R = P.r[S];
        if constexpr (PCS >= 0) {
            constexpr int nbt = (L / R) << PCS;
    #pragma unroll
            for (int t0 = 0; t0 < nbt; t0 += NT) {
                const int t = t0 + (int)threadIdx.x;
                if (nbt % NT == 0 || t < nbt)
                    stockham_butterfly_ct<T, R, L, NS, DERIV && S + 1 == P.n, PCS>(a, b, t, pcshift, tw, dir,
                                                                                inv_l);
            }
        } else {
            const int nbt = (L / R) << pcshift;
            for (int t = threadIdx.x; t < nbt; t += NT)
                stockham_butterfly_ct<T, R, L, NS, DERIV && S + 1 == P.n>(a, b, t, pcshift, tw, dir, inv_l);
        }
        __syncthreads();
        return block_fft_ct<T, L, NT, S + 1, NS * R, DERIV, PCS>(b, a, tw, pcshift, dir, inv_l);
    }
}

// Whole transform of the PC pencils held in LDS buffer a (b is scratch of the
// same size).  Returns the buffer holding the result.  Ends with a barrier.
// tw: the twiddle table (typically a copy in LDS); the plan's radices stay in
// the kernel arguments.
template <typename T>
__device__ inline C2<T>* block_fft(C2<T>* a, C2<T>* b, const FftPlan<T>& pl, const C2<T>* tw,
                                   int pcshift, int dir) {
    int Ns = 1;
    for (int s = 0; s < pl.nrad; ++s) {
        const int R = pl.rad[s];
        const int nbt = (pl.L / R) << pcshift;
        for (int t = threadIdx.x; t < nbt; t += blockDim.x)
            stockham_dispatch<T>(R, a, b, t, pl.L, pcshift, Ns, tw, dir);
        __syncthreads();
        C2<T>* tmp = a;
        a = b;
        b = tmp;
        Ns *= R;
    }
    return a;
}
#endif

// Radix plan: as many 8s as possible (keeping the rest a power of two
// product), then 4, 2, and 3.  Returns the number of radices, 0 if L is not
// of the form 2^a 3^b.
inline int make_radices(int L, int* rad) {
    int n = 0;
    int m = L;
    int p2 = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++p2;
    }
    int p3 = 0;
    while (m % 3 == 0) {
        m /= 3;
        ++p3;
    }
    if (m != 1) return 0;
    while (p2 >= 3) {
        rad[n++] = 8;
        p2 -= 3;
    }
    if (p2 == 2) rad[n++] = 4;
    if (p2 == 1) rad[n++] = 2;
    for (int i = 0; i < p3; ++i) rad[n++] = 3;
    return n;
}

}  // namespace gan
