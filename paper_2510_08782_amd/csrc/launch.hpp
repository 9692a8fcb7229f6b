// Host-side launchers of the library's kernels (one per kernel family).
// Every launcher enqueues on `st` and returns the hipError_t of the launch.
#pragma once

#include "common.hpp"

namespace gan {

// ---- semi-Lagrangian kernels (sl.hip) --------------------------------------
// Each launcher takes `spread`, a host bound on the spread of the
// displacement floors over the field (cells: floor(B) + ceil(B) for a bound
// B >= max |d|, see spread_bound), and picks the LDS window variant that
// covers it.
// max over components and points of |s_c v_c(i)| -> res[0] (FP64 reduction)
template <typename T>
hipError_t launch_velocity_max(const Dims& dm, const T* v, const double* s, double* partial,
                               double* res, hipStream_t st);
// floor(B) + ceil(B): the spread of floor(d) over displacements |d| <= B
int spread_bound(double B);
// spread_bound of the RK2 departure displacements given max |u|
int displacement_bound(double umax, int dim);
// RK2 departure displacements (index units) for velocity +v (dX, nullable) and
// -v (dY, nullable).  s[c] = h_t / h_c converts component c to cells per step;
// spread = spread_bound(max |u|).
template <typename T>
hipError_t launch_characteristics(const Dims& dm, const T* v, const double* s, int spread, T* dX,
                                  T* dY, hipStream_t st);
// Window table of a displacement field (per gather tile the floor range of its
// displacements; window_table_ints ints): the first gather over a new field
// passes table_write = 1 and records the windows it reduces, the following
// ones pass 0 and start staging at once.  Nullable (no table).
template <typename T>
long long window_table_ints(const Dims& dm);
// out = [fac *] I[src](i + disp)
template <typename T>
hipError_t launch_sl_step(const Dims& dm, const T* src, const T* disp, const T* fac, int spread,
                          T* out, hipStream_t st, int* table = nullptr, int table_write = 0);
// out = add + I[src](i + disp)   (one step of the deformation map)
template <typename T>
hipError_t launch_sl_step_add(const Dims& dm, const T* src, const T* disp, const T* add,
                              int spread, T* out, hipStream_t st, int* table = nullptr,
                              int table_write = 0);
// out = 1 + sgn h_t/2 (I[delta](i+disp) + delta) + h_t^2/2 delta I[delta](i+disp)
template <typename T>
hipError_t launch_source_factor(const Dims& dm, const T* delta, const T* disp, double ht,
                                double sgn, int spread, T* out, hipStream_t st,
                                int* table = nullptr, int table_write = 0);

// ---- reductions and vector kernels (vec.hip) -------------------------------
// Arrays are segmented: a batch of nseg independent problems stacked along the
// slowest grid axis.  Element (c, s, i) of an array sits at
// c * cstride + s * seglen + i: component c < ncomp, segment s < nseg,
// i < seglen.  A single problem is one segment.
constexpr int kMaxSeg = 64;
constexpr int kMaxGram = 66;                          // window of 64 plus two vectors
constexpr long long kGramPartialDoubles = 256 * 1024;
struct Seg {
    int nseg;
    int ncomp;
    long long seglen;
    long long cstride;
};
struct SegCoef {
    double c[kMaxSeg];
};

// Deterministic two-stage FP64 reductions; segment s's result lands in res[s]
// (device).
int reduction_blocks(long long n);
// sum (a - b)^2 ; if lam != nullptr also writes lam = b - a
template <typename T>
hipError_t launch_sumsq_diff(const T* a, const T* b, T* lam, const Seg& g, double* partial,
                             double* res, hipStream_t st);
template <typename T>
hipError_t launch_dot(const T* a, const T* b, const Seg& g, double* partial, double* res,
                      hipStream_t st);
// max |a| with NaN mapped to +inf
template <typename T>
hipError_t launch_maxabs(const T* a, const Seg& g, double* partial, double* res, hipStream_t st);
// Gram matrix of K <= kMaxGram vectors per segment: res[q nseg + s] holds
// packed upper-triangle entry q (pairs (a, b >= a) in row order) of segment
// s.  K > 8 needs a partials buffer of kGramPartialDoubles doubles and
// K (K + 1) / 2 * nseg <= kGramPartialDoubles.
template <typename T>
hipError_t launch_gram(const T* const* vecs, int K, const Seg& g, double* partial, double* res,
                       hipStream_t st);
// out = a + s[seg] b   (s: host array, one coefficient per segment)
template <typename T>
hipError_t launch_axpy(const T* a, const double* s, const T* b, T* out, const Seg& g,
                       hipStream_t st);
// out[c] = g[c] sum_j g[j] x[j] pointwise (d components of n points each)
template <typename T>
hipError_t launch_outer(const T* g, const T* x, T* out, int d, long long n, hipStream_t st);
// out = q + sum_k coef[k nseg + s] (q - x[k]) on segment s   (K <= 65; the
// NGMRES / AA update; coef: device table)
template <typename T>
hipError_t launch_combine(const T* q, const T* const* x, const double* coef, int K, T* out,
                          const Seg& g, hipStream_t st);

// det grad y per point, y = x + h D, from J[a d + b] = dD_a/dx_b (d = 2, 3;
// h[a]: cell size along component a's axis).  det (nullable) receives the
// field; per segment s: res[s] = -min, res[nseg + s] = max,
// res[2 nseg + s] = sum (det - 1), res[3 nseg + s] = sum (det - 1)^2.
template <typename T>
hipError_t launch_det_stats(const T* const* J, const double* h, int d, const Seg& g, T* det,
                            double* partial, double* res, hipStream_t st);

// ---- spectral kernels (spectral.hip) ----------------------------------------
template <typename T>
struct SpectralPlans {
    FftPlan<T> p[3];  // one plan per internal axis (length n[a])
};

// Body-force / divergence derivative along internal axis `axis`:
//   out = [out +] sum_t w[t] * G[t] * d/dx_axis F[t]   (G[t] = 1 when G == nullptr)
// for t = 0..ntime-1 (ntime <= 65); F, G are host arrays of device fields.
template <typename T>
hipError_t launch_deriv_axis(const Dims& dm, const SpectralPlans<T>& pl, int axis,
                             const T* const* F, const T* const* G, const double* w, int ntime,
                             int accumulate, T* out, hipStream_t st);
// Forward real-to-half-spectrum transform of `count` fields (count <= 3):
// in[c] (real TI, N) -> out[c] (complex TC, NH), computed in precision TC.
// skip_last: stop before the last complex pass (axis 3 - dim), which
// launch_spec_fused then runs together with a spectral operator.
template <typename TI, typename TC>
hipError_t launch_rfft(const Dims& dm, const SpectralPlans<TC>& pl, const TI* const* in,
                       C2<TC>* const* out, int count, hipStream_t st, int skip_last = 0);
// Inverse: spec[c] (overwritten) -> out[c] = scale * real(ifft) [+ add[c]]
// skip_first: start after the first complex pass (run by launch_spec_fused).
template <typename T>
hipError_t launch_irfft(const Dims& dm, const SpectralPlans<T>& pl, C2<T>* const* spec,
                        T* const* out, const T* const* add, double scale, int count,
                        hipStream_t st, int skip_first = 0);

struct SpecOpParams {
    int dim;
    int p;             // regulariser order
    double alpha;
    int leray;         // apply the Leray projection
    const double* alpha_seg;  // device, one alpha per stacked 2-D problem (nullable)
};
// gh[c] = alpha l_p vh[c] + P bh[c]   (bh may alias gh; vh is an FP64 spectrum)
template <typename T>
hipError_t launch_spec_gradient(const Dims& dm, const SpecOpParams& sp, C2<double>* const* vh,
                                C2<T>* const* bh, C2<T>* const* gh, hipStream_t st);
// sh[c] = -P gh[c] / (alpha lbar_p)   (in place allowed); keep (nullable)
// receives a second copy
template <typename T>
hipError_t launch_spec_precond(const Dims& dm, const SpecOpParams& sp, C2<T>* const* gh,
                               C2<T>* const* sh, C2<T>* const* keep, hipStream_t st);
// The last forward and the first inverse complex pass along axis 3 - dim fused
// with a pointwise operator on the sp.dim spectra io[c] (in place; between
// launch_rfft(..., skip_last = 1) and launch_irfft(..., skip_first = 1)):
//   kSpecGrad:    io = alpha l_p vh + P io      (as launch_spec_gradient)
//   kSpecPrecond: io = -P io / (alpha lbar_p)   (as launch_spec_precond; keep
//                 nullable receives a copy of the spectrum)
// kSpecGrad with keep and pre (both or neither): the preconditioned direction
// of the new gradient, -P g^ / (alpha lbar_p) over the full spectrum, goes to
// keep[c] and pre[c] (the caller transforms pre back; keep stays)
constexpr int kSpecGrad = 0, kSpecPrecond = 1;
template <typename T>
hipError_t launch_spec_fused(const Dims& dm, const SpectralPlans<T>& pl, int op,
                             const SpecOpParams& sp, C2<T>* const* io, C2<double>* const* vh,
                             C2<T>* const* keep, hipStream_t st, C2<T>* const* pre = nullptr);
// sh[c] = sign (alpha lbar_p)^expo P gh[c] (P only when sp.leray; lbar_p: l_p
// with its zero entry set to one); band_cut: the modes outside |k_i| <= n_i/2 - 1
// are set to zero.
template <typename T>
hipError_t launch_spec_pow(const Dims& dm, const SpecOpParams& sp, C2<T>* const* gh,
                           C2<T>* const* sh, double expo, double sign, int band_cut,
                           hipStream_t st);
// Half spectra between the grid df and dc (half the cells on every
// interpolated axis): to_coarse: dst (coarse) = scale src (fine) on the coarse
// space |k_i| <= dc.n_i/2 - 1, else dst (fine) = scale src (coarse) there;
// every other destination entry is zero.
template <typename T>
hipError_t launch_spec_resample(const Dims& df, const Dims& dc, C2<T>* const* src,
                                C2<T>* const* dst, int count, int to_coarse, double scale,
                                hipStream_t st);
// Per stacked problem s (one for 3-D): res[s] = sum w l_p Re(vh conj sh),
// res[nseg + s] = sum w l_p |sh|^2 (full-spectrum sums)
template <typename T>
hipError_t launch_spec_cross(const Dims& dm, const SpecOpParams& sp, C2<double>* const* vh,
                             C2<T>* const* sh, double* partial, double* res, hipStream_t st);
// vh[c] += rho[s] sh[c] on stacked problem s (rho: host array)
template <typename T>
hipError_t launch_spec_axpy(const Dims& dm, int dim, C2<double>* const* vh, const double* rho,
                            C2<T>* const* sh, hipStream_t st);
// res[s] = sum_c sum_k l_p(k) |vh_c(k)|^2 over the full spectrum of stacked
// problem s (half-spectrum weights)
template <typename T>
hipError_t launch_spec_regvalue(const Dims& dm, const SpecOpParams& sp, C2<T>* const* vh,
                                double* partial, double* res, hipStream_t st);

}  // namespace gan
