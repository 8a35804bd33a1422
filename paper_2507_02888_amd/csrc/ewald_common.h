// Device helpers shared by every kernel translation unit of libewald (gfx950):
// complex arithmetic, phases in turns, minimum-image geometry, the pair
// potential, wave reductions, phase tables and the rho rebuild, plus the
// host-side launch helpers.  Internal; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <type_traits>

#include "ewald_internal.h"

namespace ewald {


template <typename R>
struct cplx {
  R x, y;
};

// Complex product with the FMAs written out, so that every kernel and launch
// shape rounds it the same way (left to itself the compiler may contract
// either product of each component).
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}

__device__ __forceinline__ int unpack_n(uint32_t p, int d) {
  return int(int8_t((p >> (8 * d)) & 0xffu));
}

__device__ __forceinline__ double wrap01(double x) {
  double f = x - floor(x);
  return f >= 1.0 ? 0.0 : f;
}

// Cartesian row vector -> wrapped fractional coordinates.
template <int DIM>
__device__ __forceinline__ void to_frac(const double* r, const double* Ainv, double* s) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    double v = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) v = fma(r[e], Ainv[e * 3 + d], v);
    s[d] = wrap01(v);
  }
}

// exp(2 pi i x) in turns: reduce x to the nearest quarter turn q and a
// remainder of at most half a quarter turn (exact in FP64), evaluate the
// Taylor series of cos and sin at theta = remainder * pi/2 (|theta| <= pi/4;
// the first omitted terms are below 1e-19), and rotate by i^q.  Small and
// register-light, unlike a general sincos.  Both precision forms build their
// phase tables from it in FP64 (the mixed form rounds the entries to FP32).
__device__ __forceinline__ void quarter_turns(double x, double& r, int& q) {
  x -= rint(x);
  const double y = 4.0 * x;
  const double qd = rint(y);
  r = y - qd;
  q = int(qd) & 3;
}

template <typename R>
__device__ __forceinline__ cplx<R> rotate_quarter(R c, R s, int q) {
  const R x = (q & 1) ? -s : c, y = (q & 1) ? c : s;
  return (q & 2) ? cplx<R>{-x, -y} : cplx<R>{x, y};
}

__device__ __forceinline__ cplx<double> turn(double x) {
  double r;
  int q;
  quarter_turns(x, r, q);
  const double th = r * 1.5707963267948966, t2 = th * th;
  double sp = 2.8114572543455206e-15;
  sp = fma(sp, t2, -7.6471637318198165e-13);
  sp = fma(sp, t2, 1.6059043836821613e-10);
  sp = fma(sp, t2, -2.5052108385441720e-08);
  sp = fma(sp, t2, 2.7557319223985893e-06);
  sp = fma(sp, t2, -1.9841269841269841e-04);
  sp = fma(sp, t2, 8.3333333333333333e-03);
  sp = fma(sp, t2, -1.6666666666666667e-01);
  sp = fma(sp, t2 * th, th);
  double cp = -1.5619206968586225e-16;
  cp = fma(cp, t2, 4.7794773323873853e-14);
  cp = fma(cp, t2, -1.1470745597729725e-11);
  cp = fma(cp, t2, 2.0876756987868099e-09);
  cp = fma(cp, t2, -2.7557319223985891e-07);
  cp = fma(cp, t2, 2.4801587301587302e-05);
  cp = fma(cp, t2, -1.3888888888888889e-03);
  cp = fma(cp, t2, 4.1666666666666667e-02);
  cp = fma(cp, t2, -0.5);
  cp = fma(cp, t2, 1.0);
  return rotate_quarter<double>(cp, sp, q);
}

// Squared minimum-image distance between fractional positions a and b:
// reduce the fractional difference to [-1/2, 1/2], go Cartesian in the frame
// where the lattice rows are lower-triangular (Lrot; distances are frame
// independent), then compare with the candidate images r0 +- v_c
// (|r0 +- v|^2 = |r0|^2 + |v|^2 -+ 2 r0.v).
template <int DIM>
__device__ __forceinline__ double min_r2(const double* a, const double* b, const DevSys* __restrict__ S,
                                         int n_cand) {
  double f[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    f[d] = a[d] - b[d];
    f[d] -= rint(f[d]);
  }
  const double* L = S->Lrot;
  double r[DIM];
  if constexpr (DIM == 3) {
    r[0] = fma(f[2], L[6], fma(f[1], L[3], f[0] * L[0]));
    r[1] = fma(f[2], L[7], f[1] * L[4]);
    r[DIM - 1] = f[DIM - 1] * L[8];
  } else {
    r[0] = fma(f[1], L[3], f[0] * L[0]);
    r[DIM - 1] = f[DIM - 1] * L[4];
  }
  double r0sq = 0.0;
#pragma unroll
  for (int e = 0; e < DIM; ++e) r0sq = fma(r[e], r[e], r0sq);
  double r2 = r0sq;
  for (int c = 0; c < n_cand; ++c) {
    double dot = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) dot = fma(r[e], S->cand[c][e], dot);
    r2 = fmin(r2, fma(-2.0, fabs(dot), r0sq + S->cand[c][3]));
  }
  return r2;
}

// Squared minimum-image distance in the orthogonal-sublattice frame: wrap
// each axis into the box (|x_d| <= box_d / 2); the nearest image in the coset
// offset by half box sides along the axes of its mask is at
// sum_mask (box_d/2 - |x_d|)^2 + sum_other x_d^2 = |x|^2 + cc - sum_d cw_d |x_d|
// (cw_d = box_d on the mask, else 0; cc = +inf when the frame has no coset,
// so the expression needs no branch).
// The constants a pair distance and a pair term need, by value: for kernels
// with vector registers to spare they are loaded once into vector registers
// (frame_k_vector), elsewhere read from the system tables (frame_k).
struct FrameK {
  double box[3], ibox[3], cw[3], cc;
  double rc2, alpha, scale;  // r_cut^2, alpha, 2 / r_cut^2 (pair potential)
};

__device__ __forceinline__ FrameK frame_k(const DevSys* __restrict__ S) {
  FrameK K;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    K.box[d] = S->box[d];
    K.ibox[d] = S->ibox[d];
    K.cw[d] = S->cw[0][d];
  }
  K.cc = S->cc[0];
  K.rc2 = S->rc2;
  K.alpha = S->alpha;
  K.scale = S->poly_scale;
  return K;
}

// Loaded with a lane-varying index, so that the compiler keeps them in vector
// registers rather than in the scarcer scalar ones.
__device__ __forceinline__ FrameK frame_k_vector(const DevSys* __restrict__ S) {
  int z = 0;
  asm volatile("" : "+v"(z));
  FrameK K;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    K.box[d] = S->box[d + z];
    K.ibox[d] = S->ibox[d + z];
    K.cw[d] = S->cw[0][d + z];
  }
  K.cc = S->cc[z];
  K.rc2 = (&S->rc2)[z];
  K.alpha = (&S->alpha)[z];
  K.scale = (&S->poly_scale)[z];
  return K;
}

template <int DIM>
__device__ __forceinline__ double min_r2_ortho(const double* a, const double* b, const FrameK& K) {
  double x[DIM], r0sq = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    x[d] = a[d] - b[d];
    x[d] = fma(-K.box[d], rint(x[d] * K.ibox[d]), x[d]);
    r0sq = fma(x[d], x[d], r0sq);
  }
  double t = r0sq + K.cc;
#pragma unroll
  for (int d = 0; d < DIM; ++d) t = fma(-K.cw[d], fabs(x[d]), t);
  return fmin(r0sq, t);
}

// A reference to one of two arrays chosen at compile time.
template <bool B, typename A, typename C>
__device__ __forceinline__ auto& pick_ref(A& a, C& c) {
  if constexpr (B)
    return c;
  else
    return a;
}

// Coordinates of a fractional position in the orthogonal-sublattice frame.
template <int DIM>
__device__ __forceinline__ void frame_coords(const double* s, const DevSys* __restrict__ S, double* x) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) v = fma(s[i], S->F[i * 3 + d], v);
    x[d] = v;
  }
}

// Minimum-image r^2 between two positions given in the kernel's geometry:
// frame coordinates (ORTHO) or fractional coordinates (general cells).
template <int DIM, bool ORTHO>
__device__ __forceinline__ double image_r2(const double* a, const double* b, const DevSys* __restrict__ S,
                                           int n_cand, const FrameK& K) {
  if (ORTHO) return min_r2_ortho<DIM>(a, b, K);
  return min_r2<DIM>(a, b, S, n_cand);
}

// A stored (fractional) position in the kernel's geometry.
template <int DIM, bool ORTHO>
__device__ __forceinline__ void geo_pos(const double* s, const DevSys* __restrict__ S, double* x) {
  if (ORTHO) {
    frame_coords<DIM>(s, S, x);
  } else {
#pragma unroll
    for (int d = 0; d < DIM; ++d) x[d] = s[d];
  }
}

// A value every lane holds alike (read from LDS at a uniform address), made
// visibly uniform for the compiler: scalar registers, and branches on it
// stay branches (not per-lane selects).
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform_d(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform_r(double v) { return uniform_d(v); }
__device__ __forceinline__ float uniform_r(float v) { return uniform_f(v); }

// Kahan-compensated FP32 accumulator.
struct Kahan {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float v) {
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ double value() const { return double(s) - double(c); }
};

// Pair potential phi(r) = erfc(alpha r)/r = 1/r - alpha g(alpha^2 r^2) for
// r^2 < rc2, where g(y) = erf(sqrt y)/sqrt y is entire.  On [0, r_cut] g is
// one polynomial in t = 2 r^2 / r_cut^2 - 1 (degree PD, fitted in FP64 by the
// set-up), so a pair costs one reciprocal square root and PD FMAs.
// FP64 form: everything in FP64.  Mixed form: 1/r in FP64 (it carries the
// close-pair singularity) and the bounded erf part in FP32 (degree 12 or 22)
// summed with Kahan compensation.
template <bool MIXED, int PD>
struct PairAcc;

// 1/sqrt(x) for x in (0, r_cut^2]: the hardware estimate refined by one
// Newton step carried to second order, y (1 + e/2 + 3e^2/8) with
// e = 1 - x y^2 (remaining relative error ~5e^3/16).  Unlike the library
// rsqrt it has no zero/infinity/denormal handling, which the pair terms never
// need (coincident particles are documented as giving non-finite results).
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// Pair terms are evaluated several at a time (NE = 2 or 4): the four Horner chains interleave
// (latency hiding) and take their coefficients straight from scalar registers.
// A term enters iff r2 < r_cut^2; callers pad with r2 = r_cut^2 and q = 0.
template <int PD>
struct PairAcc<false, PD> {
  double s = 0.0;
  const double* __restrict__ c;  // the polynomial coefficients (system tables, or registers)
  const FrameK& K;
  __device__ __forceinline__ PairAcc(const double* c64, const float*, const FrameK& k) : c(c64), K(k) {}
  template <int NE>
  __device__ __forceinline__ void add(const double (&q)[NE], const double (&r2)[NE]) {
    double ir[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) ir[e] = rsqrt_pos(r2[e]);
    add_ir<NE>(q, r2, ir);
  }
  // the same with 1/sqrt(r2) already formed (shared with the Jastrow u term)
  template <int NE>
  __device__ __forceinline__ void add_ir(const double (&q)[NE], const double (&r2)[NE], const double (&ir)[NE]) {
    double t[NE], p[NE];
    const double scale = K.scale;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      t[e] = fma(r2[e], scale, -1.0);
      p[e] = c[PD];
    }
#pragma unroll
    for (int i = PD - 1; i >= 0; --i) {
      const double ci = c[i];
#pragma unroll
      for (int e = 0; e < NE; ++e) p[e] = fma(p[e], t[e], ci);
    }
    const double rc2 = K.rc2, alpha = K.alpha;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const double phi = fma(-alpha, p[e], ir[e]);
      s = fma(r2[e] < rc2 ? q[e] : 0.0, phi, s);
    }
  }
  __device__ __forceinline__ double value() const { return s; }
};

template <int PD>
struct PairAcc<true, PD> {
  static constexpr int PF = PD == 16 ? 12 : 22;
  double inv = 0.0;
  Kahan erfpart;
  const float* __restrict__ c;  // the FP32 polynomial coefficients (system tables, or registers)
  const FrameK& K;
  __device__ __forceinline__ PairAcc(const double*, const float* c32, const FrameK& k) : c(c32), K(k) {}
  template <int NE>
  __device__ __forceinline__ void add(const double (&q)[NE], const double (&r2)[NE]) {
    double ir[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) ir[e] = rsqrt_pos(r2[e]);
    add_ir<NE>(q, r2, ir);
  }
  template <int NE>
  __device__ __forceinline__ void add_ir(const double (&q)[NE], const double (&r2)[NE], const double (&ir)[NE]) {
    float t[NE], p[NE];
    const float scale = float(K.scale);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      t[e] = fmaf(float(r2[e]), scale, -1.0f);
      p[e] = c[PF];
    }
#pragma unroll
    for (int i = PF - 1; i >= 0; --i) {
      const float ci = c[i];
#pragma unroll
      for (int e = 0; e < NE; ++e) p[e] = fmaf(p[e], t[e], ci);
    }
    const double rc2 = K.rc2;
    const float alpha = float(K.alpha);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const double qe = r2[e] < rc2 ? q[e] : 0.0;
      inv = fma(qe, ir[e], inv);
      erfpart.add(float(qe) * (alpha * p[e]));
    }
  }
  __device__ __forceinline__ double value() const { return inv - erfpart.value(); }
};

// ---------------------------------------------------------------------------
// Jastrow two-body polynomial term u (Sec. 2.3, Eq. (8)), in powers of
// t = r / L_u with the coefficients of the pair's spin channel,
// c_m = u_c0[m] + s u_dc[m] (s = 0 for equal labels, 1 for unequal ones).
// FP64 in both precision forms.

// u at two arguments (a moved particle's new and old position against one
// partner), sharing the channel blend.
__device__ __forceinline__ void u_two(const DevSys* __restrict__ S, double s, double ta, double tb, double& ua,
                                      double& ub) {
  double pa = 0.0, pb = 0.0;
#pragma unroll
  for (int m = UDEG; m >= 0; --m) {
    const double c = fma(s, S->u_dc[m], S->u_c0[m]);
    pa = fma(pa, ta, c);
    pb = fma(pb, tb, c);
  }
  ua = pa;
  ub = pb;
}

// u and its first and second derivatives with respect to t at one argument,
// and u at a second one (Horner with derivative chains).
__device__ __forceinline__ void u_der_two(const DevSys* __restrict__ S, double s, double ta, double tb, double& ua,
                                          double& d1, double& d2, double& ub) {
  double p = 0.0, p1 = 0.0, p2 = 0.0, pb = 0.0;
#pragma unroll
  for (int m = UDEG; m >= 0; --m) {
    const double c = fma(s, S->u_dc[m], S->u_c0[m]);
    p2 = fma(p2, ta, p1);
    p1 = fma(p1, ta, p);
    p = fma(p, ta, c);
    pb = fma(pb, tb, c);
  }
  ua = p;
  d1 = p1;
  d2 = 2.0 * p2;
  ub = pb;
}

// u of one pair at r^2 with 1/r given (energy sums); 0 beyond L_u or when
// the pair does not take part.
__device__ __forceinline__ double u_pair(const DevSys* __restrict__ S, bool take, bool unequal, double r2,
                                         double ir) {
  double u, unused;
  u_two(S, unequal ? 1.0 : 0.0, r2 * ir * S->u_icut, 0.0, u, unused);
  return (take && r2 < S->u_cut2) ? u : 0.0;
}

// Change of U in a move against one partner (new minus old), and for UD the
// partner's share of grad_k U (in the geometry's frame axes: x is the
// minimum-image displacement of the new position from the partner) and of
// lap_k U at the new position.
template <int DIM>
struct UOut {
  double d = 0.0;
  double g[DIM] = {};
  double l = 0.0;
};

template <int DIM, bool UD>
__device__ __forceinline__ void u_move_term(const DevSys* __restrict__ S, bool ok, bool unequal, double r2n,
                                            double irn, double r2o, double iro, const double* xn, UOut<DIM>& out) {
  const double s = unequal ? 1.0 : 0.0, ic = S->u_icut, uc2 = S->u_cut2;
  const double tn = r2n * irn * ic, to = r2o * iro * ic;
  const bool inn = ok && r2n < uc2, ino = ok && r2o < uc2;
  double un, uo;
  if (UD) {
    double d1, d2;
    u_der_two(S, s, tn, to, un, d1, d2, uo);
    const double dur = inn ? d1 * ic * irn : 0.0;  // u'(r) / r
#pragma unroll
    for (int d = 0; d < DIM; ++d) out.g[d] = fma(dur, xn[d], out.g[d]);
    out.l += inn ? fma(d2, ic * ic, double(DIM - 1) * dur) : 0.0;
  } else {
    u_two(S, s, tn, to, un, uo);
  }
  out.d += (inn ? un : 0.0) - (ino ? uo : 0.0);
}

// A vector in a frame's axes (rows of E) in Cartesian axes.
template <int DIM>
__device__ __forceinline__ void frame_to_cart(const double* x, const double* E, double* out) {
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    double v = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) v = fma(x[d], E[d * 3 + e], v);
    out[e] = v;
  }
}

// Minimum-image displacement a - b (as min_r2, which gives the same r^2) in
// the lower-triangular frame's axes; returns r^2.
template <int DIM>
__device__ __forceinline__ double min_disp(const double* a, const double* b, const DevSys* __restrict__ S,
                                           int n_cand, double* x) {
  double f[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    f[d] = a[d] - b[d];
    f[d] -= rint(f[d]);
  }
  const double* L = S->Lrot;
  double r[DIM];
  if constexpr (DIM == 3) {
    r[0] = fma(f[2], L[6], fma(f[1], L[3], f[0] * L[0]));
    r[1] = fma(f[2], L[7], f[1] * L[4]);
    r[DIM - 1] = f[DIM - 1] * L[8];
  } else {
    r[0] = fma(f[1], L[3], f[0] * L[0]);
    r[DIM - 1] = f[DIM - 1] * L[4];
  }
  double r0sq = 0.0;
#pragma unroll
  for (int e = 0; e < DIM; ++e) r0sq = fma(r[e], r[e], r0sq);
  double r2 = r0sq;
#pragma unroll
  for (int e = 0; e < DIM; ++e) x[e] = r[e];
  for (int c = 0; c < n_cand; ++c) {
    double dot = 0.0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) dot = fma(r[e], S->cand[c][e], dot);
    const double t = fma(-2.0, fabs(dot), r0sq + S->cand[c][3]);
    if (t < r2) {
      r2 = t;
      const double sg = dot >= 0.0 ? 1.0 : -1.0;
#pragma unroll
      for (int e = 0; e < DIM; ++e) x[e] = fma(-sg, S->cand[c][e], r[e]);
    }
  }
  return r2;
}

// The same in the orthogonal-sublattice frame (as min_r2_ortho): the coset
// image moves each masked axis by half a box side towards zero.
template <int DIM>
__device__ __forceinline__ double min_disp_ortho(const double* a, const double* b, const FrameK& K, double* x) {
  double r0sq = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    x[d] = a[d] - b[d];
    x[d] = fma(-K.box[d], rint(x[d] * K.ibox[d]), x[d]);
    r0sq = fma(x[d], x[d], r0sq);
  }
  double t = r0sq + K.cc;
#pragma unroll
  for (int d = 0; d < DIM; ++d) t = fma(-K.cw[d], fabs(x[d]), t);
  if (t < r0sq) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) x[d] -= copysign(0.5 * K.cw[d], x[d]);
    return t;
  }
  return r0sq;
}

template <int DIM, bool ORTHO>
__device__ __forceinline__ double image_disp(const double* a, const double* b, const DevSys* __restrict__ S,
                                             int n_cand, const FrameK& K, double* x) {
  if (ORTHO) return min_disp_ortho<DIM>(a, b, K, x);
  return min_disp<DIM>(a, b, S, n_cand, x);
}

// Real-space part of a move of particle k from so to sn, summed over the
// mobile particles j != k (positions pos, charges q) and the fixed ions:
// sum_j q_j [phi(sn - s_j) - phi(so - s_j)].  Threads take j = tid, tid + NT, ...
// PPR particles (2 PPR pair terms) per round: 2 for workgroups of up to 512
// threads, 1 for 1024 (one particle per thread at N = 1024).  Indices are
// clamped rather than branched on, so every load is in bounds and the loop
// body has no divergent control flow.  UJ: also the Jastrow u term of the
// mobile pairs into uo (UD: with its gradient, in the lower-triangular
// frame's axes, and Laplacian at the new position).
// A layered 2D system (S->n_layers = 2) adds (z_1 - z_0)^2 to r^2 for the
// partners in the other plane.  sub_k >= 0: particle sub_k is taken at
// sub_s instead of its stored position (a move accepted in the same launch).
template <int DIM, bool MIXED, int PD, int NT, bool UJ = false, bool UD = false>
__device__ __forceinline__ double real_move(const double* sn, const double* so, int k, const double* pos,
                                            const double* q, int n, const DevSys* __restrict__ S,
                                            UOut<DIM>* uo = nullptr, int sub_k = -1,
                                            const double* sub_s = nullptr) {
  constexpr int PPR = NT >= 1024 ? 1 : 2;
  const FrameK K = frame_k(S);
  PairAcc<MIXED, PD> pr(S->p64, S->p32, K);
  const int n_cand = S->n_cand;
  const double rc2 = S->rc2;
  const int sk = UJ ? S->spin[k] : 0;
  const bool lay = DIM == 2 && S->n_layers > 1;
  const int n0 = S->n0, lk = k >= n0 ? 1 : 0;
  const double dz2 = S->dz2;
  for (int j0 = threadIdx.x; j0 < n; j0 += PPR * NT) {
    double qq[2 * PPR], r2[2 * PPR], ir[2 * PPR];
    double xn[UD ? PPR : 1][DIM] = {};  // zero for masked partners (their weight is zero too)
    bool okc[PPR];
    int sj[PPR];
#pragma unroll
    for (int c = 0; c < PPR; ++c) {
      const int j = j0 + c * NT;
      const bool ok = j < n && j != k;
      const int jj = j < n ? j : n - 1;
      double pj[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) pj[d] = jj == sub_k ? sub_s[d] : pos[jj * DIM + d];
      const double qj = ok ? q[jj] : 0.0;
      if (UD)
        r2[2 * c] = ok ? min_disp<DIM>(sn, pj, S, n_cand, xn[UD ? c : 0]) : rc2;
      else
        r2[2 * c] = ok ? min_r2<DIM>(sn, pj, S, n_cand) : rc2;
      r2[2 * c + 1] = ok ? min_r2<DIM>(so, pj, S, n_cand) : rc2;
      if (lay && ok && (jj >= n0 ? 1 : 0) != lk) {
        r2[2 * c] += dz2;
        r2[2 * c + 1] += dz2;
      }
      qq[2 * c] = qj;
      qq[2 * c + 1] = -qj;
      okc[c] = ok;
      if (UJ) sj[c] = S->spin[jj];
    }
#pragma unroll
    for (int e = 0; e < 2 * PPR; ++e) ir[e] = rsqrt_pos(r2[e]);
    pr.template add_ir<2 * PPR>(qq, r2, ir);
    if (UJ)
#pragma unroll
      for (int c = 0; c < PPR; ++c)
        u_move_term<DIM, UD>(S, okc[c], sj[c] != sk, r2[2 * c], ir[2 * c], r2[2 * c + 1], ir[2 * c + 1],
                             xn[UD ? c : 0], *uo);
  }
  const int nfix = S->n_fixed;
  for (int j0 = threadIdx.x; j0 < nfix; j0 += PPR * NT) {
    double qq[2 * PPR], r2[2 * PPR];
#pragma unroll
    for (int c = 0; c < PPR; ++c) {
      const int j = j0 + c * NT;
      const bool ok = j < nfix;
      const int jj = ok ? j : nfix - 1;
      double sj[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) sj[d] = S->fixed_s[jj * DIM + d];
      const double qj = ok ? S->fixed_q[jj] : 0.0;
      r2[2 * c] = ok ? min_r2<DIM>(sn, sj, S, n_cand) : rc2;
      r2[2 * c + 1] = ok ? min_r2<DIM>(so, sj, S, n_cand) : rc2;
      if (lay && ok && S->fixed_layer[jj] != lk) {
        r2[2 * c] += dz2;
        r2[2 * c + 1] += dz2;
      }
      qq[2 * c] = qj;
      qq[2 * c + 1] = -qj;
    }
    pr.template add<2 * PPR>(qq, r2);
  }
  return pr.value();
}

// Real-space part of a move inside the fused sweep.  Thread t owns the
// particles j = t + c NT (c < PPR) and keeps their positions (in the
// kernel's geometry: frame or fractional coordinates, as sn and so) and
// charges in registers (ps, pq); it alone updates them when they move.  Particles beyond
// PPR NT (larger systems than the launch shape covers) are read from the LDS
// copy, again only by their owner t = j mod NT.  XTRA = false: the batch has
// no such particles and no fixed ions, and those loops are left out (at 1024
// threads their mere presence costs scalar-register reloads on every move).
// UJ: also the Jastrow u term of the mobile pairs into uo (psp: the spin
// labels of the thread's own particles, sk: the moved particle's); UD: with
// its gradient (in the geometry's frame axes) and Laplacian at the new
// position.
// LAY (a layered system when `lay`): partners in the other plane (mobile
// j >= n0 against k, or an ion's plane) are dz2 further apart in r^2.
template <int DIM, bool MIXED, int PD, int NT, int PPR, bool ORTHO, bool XTRA, bool UJ = false, bool UD = false,
          bool LAY = false>
__device__ __forceinline__ double real_move_own(const double* sn, const double* so, int k,
                                                const double (&ps)[PPR][DIM], const double (&pq)[PPR],
                                                const double* lpos, const double* lq, int n,
                                                const DevSys* __restrict__ S, const double* c64,
                                                const float* c32, const FrameK& K,
                                                const int* psp = nullptr, int sk = 0,
                                                UOut<DIM>* uo = nullptr, bool lay = false, int n0 = 0,
                                                double dz2 = 0.0) {
  PairAcc<MIXED, PD> pr(c64, c32, K);
  const int n_cand = S->n_cand;
  const double rc2 = S->rc2;
  const int lk = k >= n0 ? 1 : 0;
  // the own particles c < NC; a wave evaluates only the c for which some
  // lane holds a particle (the count is the same for every lane of the
  // wave), so small walkers in a large workgroup skip the empty ones
  auto own = [&](auto nc) {
    constexpr int NC = decltype(nc)::value;
    double qq[2 * NC], r2[2 * NC], ir[2 * NC];
    double xn[UD ? NC : 1][DIM] = {};  // zero for masked partners (their weight is zero too)
    bool okc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = threadIdx.x + c * NT;
      const bool ok = j < n && j != k;
      if (UD)
        r2[2 * c] = ok ? image_disp<DIM, ORTHO>(sn, ps[c], S, n_cand, K, xn[UD ? c : 0]) : rc2;
      else
        r2[2 * c] = ok ? image_r2<DIM, ORTHO>(sn, ps[c], S, n_cand, K) : rc2;
      r2[2 * c + 1] = ok ? image_r2<DIM, ORTHO>(so, ps[c], S, n_cand, K) : rc2;
      if (LAY && lay && ok && (j >= n0 ? 1 : 0) != lk) {
        r2[2 * c] += dz2;
        r2[2 * c + 1] += dz2;
      }
      qq[2 * c] = pq[c];
      qq[2 * c + 1] = -pq[c];
      okc[c] = ok;
    }
#pragma unroll
    for (int e = 0; e < 2 * NC; ++e) ir[e] = rsqrt_pos(r2[e]);
    pr.template add_ir<2 * NC>(qq, r2, ir);
    if (UJ)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        u_move_term<DIM, UD>(S, okc[c], psp[c] != sk, r2[2 * c], ir[2 * c], r2[2 * c + 1], ir[2 * c + 1],
                             xn[UD ? c : 0], *uo);
  };
  static_assert(PPR == 1 || PPR == 2, "own particles per thread: 1 or 2");
  {
    const int wbase = uniform_i(int(threadIdx.x) & ~63);  // the wave's first thread
    const int cw = n > wbase ? min(PPR, (n - wbase + NT - 1) / NT) : 0;
    if (cw >= PPR)
      own(std::integral_constant<int, PPR>{});
    else if (PPR > 1 && cw == 1)
      own(std::integral_constant<int, 1>{});
  }
  if (!XTRA) return pr.value();
  for (int j = threadIdx.x + PPR * NT; j < n; j += NT) {
    double qq[2], r2[2], ir[2];
    double xn[DIM] = {};
    const bool ok = j != k;
    double xj[DIM];
    geo_pos<DIM, ORTHO>(lpos + j * DIM, S, xj);
    if (UD)
      r2[0] = ok ? image_disp<DIM, ORTHO>(sn, xj, S, n_cand, K, xn) : rc2;
    else
      r2[0] = ok ? image_r2<DIM, ORTHO>(sn, xj, S, n_cand, K) : rc2;
    r2[1] = ok ? image_r2<DIM, ORTHO>(so, xj, S, n_cand, K) : rc2;
    if (LAY && lay && ok && (j >= n0 ? 1 : 0) != lk) {
      r2[0] += dz2;
      r2[1] += dz2;
    }
    qq[0] = lq[j];
    qq[1] = -lq[j];
    ir[0] = rsqrt_pos(r2[0]);
    ir[1] = rsqrt_pos(r2[1]);
    pr.template add_ir<2>(qq, r2, ir);
    if (UJ) u_move_term<DIM, UD>(S, ok, S->spin[j] != sk, r2[0], ir[0], r2[1], ir[1], xn, *uo);
  }
  const int nfix = S->n_fixed;
  for (int j0 = threadIdx.x; j0 < nfix; j0 += 2 * NT) {
    double qq[4], r2[4];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int j = j0 + c * NT;
      const bool ok = j < nfix;
      const int jj = ok ? j : nfix - 1;
      double sj[DIM];
      geo_pos<DIM, ORTHO>(S->fixed_s + jj * DIM, S, sj);
      const double qj = ok ? S->fixed_q[jj] : 0.0;
      r2[2 * c] = ok ? image_r2<DIM, ORTHO>(sn, sj, S, n_cand, K) : rc2;
      r2[2 * c + 1] = ok ? image_r2<DIM, ORTHO>(so, sj, S, n_cand, K) : rc2;
      if (LAY && lay && ok && S->fixed_layer[jj] != lk) {
        r2[2 * c] += dz2;
        r2[2 * c + 1] += dz2;
      }
      qq[2 * c] = qj;
      qq[2 * c + 1] = -qj;
    }
    pr.template add<4>(qq, r2);
  }
  return pr.value();
}

// Sum NV values over a workgroup of NT threads; the result is valid in
// thread 0.  red must hold NV * NT / 64 doubles.
template <int NV, int NT = BLOCK>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * (NT / 64) + wv] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < NT / 64; ++k) t += red[i * (NT / 64) + k];
      v[i] = t;
    }
}

// Wave64 sum with DPP row operations (no LDS round trips); the total lands in
// lane 63.  Steps: swap neighbours, swap pairs, mirror half rows, mirror rows
// (every lane of a row then holds the row sum), then add row 0 into row 1 and
// row 2 into row 3 (row_bcast15), and rows 0-1 into rows 2-3 (row_bcast31).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_take(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over each row of 16 lanes with DPP moves whose every lane has a source
// (no previous value to preserve); every lane of a row ends with the row sum.
template <int CTRL>
__device__ __forceinline__ double dpp_all(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_all<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_all<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_all<0x141>(v);  // row_half_mirror
  v += dpp_all<0x140>(v);  // row_mirror
  return v;
}

__device__ __forceinline__ double wave_sum_to_lane63(double v) {
  v += dpp_take<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_take<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_take<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_take<0x140, 0xF>(v);  // row_mirror
  v += dpp_take<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
  v += dpp_take<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3
  return v;
}

// Phase tables: per dimension d one row of tbl = 2 nm + 1 complex entries,
// exp(2 pi i n s_d) at [nm + n] for n = -nm..nm; a table of one position is
// DIM rows.
template <typename R>
__device__ __forceinline__ cplx<R> tab_at(const cplx<R>* tab, int row, int idx, int tbl) {
  return tab[row * tbl + idx];
}

// FP64 entries as one 16-byte read (every table base in LDS is 16-byte aligned).
__device__ __forceinline__ cplx<double> ld_entry(const cplx<double>* tab, int i) {
  const double2 v = reinterpret_cast<const double2*>(tab)[i];
  return {v.x, v.y};
}

template <>
__device__ __forceinline__ cplx<double> tab_at<double>(const cplx<double>* tab, int row, int idx, int tbl) {
  return ld_entry(tab, row * tbl + idx);
}

// FP32 entries as one 8-byte read.
template <>
__device__ __forceinline__ cplx<float> tab_at<float>(const cplx<float>* tab, int row, int idx, int tbl) {
  const float2 v = reinterpret_cast<const float2*>(tab)[row * tbl + idx];
  return {v.x, v.y};
}

// An entry at a byte offset into a 16-byte aligned LDS table, as one read.
template <typename R>
__device__ __forceinline__ cplx<R> ld_at_byte(const cplx<R>* tab, uint32_t byte_off) {
  using V = typename std::conditional<sizeof(R) == 8, double2, float2>::type;
  const V v = *reinterpret_cast<const V*>(reinterpret_cast<const char*>(tab) + byte_off);
  return {v.x, v.y};
}

// One row, by one thread: powers of exp(2 pi i s) formed by repeated FP64
// multiplication (the paper's buffered powers, Sec. 5.2), with an exact
// restart every 8 powers so the rounding error stays below ~8 ulp; stored in R.
template <typename R>
__device__ __forceinline__ void fill_row(cplx<R>* row, double s, int nm) {
  const cplx<double> u = turn(s);
  cplx<double> c = {1.0, 0.0};
  row[nm] = {R(1), R(0)};
  for (int m = 1; m <= nm; ++m) {
    c = (m & 7) == 0 ? turn(double(m) * s) : cmul(c, u);
    row[nm + m] = {R(c.x), R(c.y)};
    row[nm - m] = {R(c.x), R(-c.y)};
  }
}

// The same row in FP64, every entry multiplied by `scale` (a particle's charge
// carried by its first row, so that the products of its rows include it),
// entry k stored at row[k * stride].
__device__ __forceinline__ void fill_row_scaled(cplx<double>* row, double s, int nm, double scale, int stride) {
  const cplx<double> u = turn(s);
  cplx<double> c = {1.0, 0.0};
  row[nm * stride] = {scale, 0.0};
  for (int m = 1; m <= nm; ++m) {
    c = (m & 7) == 0 ? turn(double(m) * s) : cmul(c, u);
    row[(nm + m) * stride] = {c.x * scale, c.y * scale};
    row[(nm - m) * stride] = {c.x * scale, -c.y * scale};
  }
}

// Coordinate r of (a, b) read as one array of 2 DIM values, with the index
// resolved by selects (a runtime index into register arrays would place
// them in scratch memory).
template <int DIM>
__device__ __forceinline__ double pick_coord(const double (&a)[DIM], const double (&b)[DIM], int r) {
  double v = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    v = r == d ? a[d] : v;
    v = r == DIM + d ? b[d] : v;
  }
  return v;
}

// First phase of segment `pn` from the tables.
template <int DIM, typename R>
__device__ __forceinline__ cplx<R> anchor(const cplx<R>* tab, uint32_t pn, int nm) {
  const int tbl = 2 * nm + 1;
  cplx<R> e = cmul(tab_at(tab, 0, nm + unpack_n(pn, 0), tbl), tab_at(tab, 1, nm + unpack_n(pn, 1), tbl));
  if (DIM == 3) e = cmul(e, tab_at(tab, 2, nm + unpack_n(pn, 2), tbl));
  return e;
}

// Phases along a segment: e_0 = the anchor, e_1 = e_0 u, then the three-term
// recurrence e_{j+1} = 2 Re(u) e_j - e_{j-1} for u = exp(2 pi i s_last)
// (|u| = 1): two FMAs per slot instead of a complex multiply.  Rounding errors
// grow at most linearly along the segment (they propagate through Chebyshev
// polynomials of the second kind, |U_j(cos phi)| <= j + 1).
template <typename R>
struct SegWalk {
  cplx<R> cur, prev;
  R c2;
  cplx<R> u;
  __device__ __forceinline__ SegWalk(cplx<R> a, cplx<R> u_) : cur(a), prev(a), c2(R(2) * u_.x), u(u_) {}
  // u_ and c2_ = 2 Re u_ precomputed (e.g. wave-uniform, in scalar registers)
  __device__ __forceinline__ SegWalk(cplx<R> a, cplx<R> u_, R c2_) : cur(a), prev(a), c2(c2_), u(u_) {}
  __device__ __forceinline__ void step(int j) {  // e_j -> e_{j+1}; j is a compile-time index in unrolled loops
    if (j == 0) {
      prev = cur;
      cur = cmul(cur, u);
    } else {
      const cplx<R> nx = {fma(c2, cur.x, -prev.x), fma(c2, cur.y, -prev.y)};
      prev = cur;
      cur = nx;
    }
  }
};

// Rebuild rho over the segments segs[i] = seg0 + i * NT (i < NS) of one
// walker in FP64: rho = rho_fix + sum_p q_p exp(i G.r_p), particles taken
// `tile` at a time through LDS phase tables (tabs: tile * DIM * (2nm+1)).
// The first row of each particle's tables carries its charge, so a segment's
// anchor already holds q_p exp(i G.r_p) and the walk along the segment (a
// linear recurrence) keeps the factor.  Two particles per pass give two
// independent chains; a pass reads all its table entries before its
// arithmetic.  `pos` and `q` may point to global or LDS memory.  All NT
// threads must call it.
// rfix: the fixed ions' part to start from (NULL: S->rho_fix; a layered
// system's second plane passes S->rho_fix1).
template <int DIM, int NS, int NT = BLOCK>
__device__ void rebuild_rho(cplx<double> (&acc)[NS][SEG], const uint32_t (&an)[NS], int seg0,
                            const DevSys* __restrict__ S, const double* pos, const double* q, int n,
                            cplx<double>* tabs, int tile = TILE_P, const double* rfix = nullptr) {
  const int nseg = S->n_seg, nm = S->nm, tbl = 2 * nm + 1, pstride = DIM * tbl;
  // tile layout: the tables of particles 2k and 2k + 1 interleaved entry by
  // entry, so that a pass reads both particles' entries at one address and
  // the next 16 bytes; entry (p, d, idx) at ((p / 2) pstride + d tbl + idx) 2 + p % 2
  int off[NS][DIM];  // 2 x the anchor's entry in each row of one particle's tables
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int s = seg0 + i * NT;
#pragma unroll
    for (int d = 0; d < DIM; ++d) off[i][d] = 2 * (d * tbl + nm + unpack_n(an[i], d));
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      if (s < nseg) {
        const double* rf = (rfix ? rfix : S->rho_fix) + 2 * (size_t(j) * nseg + s);
        acc[i][j] = {rf[0], rf[1]};
      } else {
        acc[i][j] = {0.0, 0.0};
      }
    }
  }
  auto base = [&](int p) { return tabs + (p >> 1) * (2 * pstride) + (p & 1); };
  auto entries = [&](int i, int p, cplx<double> (&e)[DIM]) {
    const cplx<double>* t = base(p);
#pragma unroll
    for (int d = 0; d < DIM; ++d) e[d] = ld_entry(t, off[i][d]);
  };
  auto product = [](const cplx<double> (&e)[DIM]) {
    cplx<double> v = cmul(e[0], e[1]);
    if (DIM == 3) v = cmul(v, e[DIM - 1]);
    return v;
  };
  for (int p0 = 0; p0 < n; p0 += tile) {  // tile is even
    const int np = min(tile, n - p0);
    for (int e = threadIdx.x; e < np * DIM; e += NT) {  // row e: particle e / DIM, dimension e % DIM
      const int pp = e / DIM, d = e - pp * DIM;
      fill_row_scaled(base(pp) + 2 * d * tbl, pos[p0 * DIM + e], nm, d == 0 ? q[p0 + pp] : 1.0, 2);
    }
    __syncthreads();
    // the step phase exp(2 pi i s_last) of a particle is one entry of its
    // tables, read by every lane at the same address (an LDS broadcast)
    auto step_phase = [&](int p) { return ld_entry(base(p), 2 * ((DIM - 1) * tbl + nm + 1)); };
    const int npair = np >> 1;
    // one pass: the pair (p, p + 1) with the entries a (particle p) and b
    auto pass = [&](int i, int p, const cplx<double> (&a)[DIM], const cplx<double> (&b)[DIM]) {
      if (seg0 + i * NT < nseg) {
        SegWalk<double> w0(product(a), step_phase(p)), w1(product(b), step_phase(p + 1));
#pragma unroll
        for (int j = 0; j < SEG; ++j) {
          acc[i][j].x = (acc[i][j].x + w0.cur.x) + w1.cur.x;
          acc[i][j].y = (acc[i][j].y + w0.cur.y) + w1.cur.y;
          if (j + 1 < SEG) {
            w0.step(j);
            w1.step(j);
          }
        }
      }
    };
    for (int pr = 0; pr < npair; ++pr)
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        cplx<double> a0[DIM], b0[DIM];
        entries(i, 2 * pr, a0);
        entries(i, 2 * pr + 1, b0);
        pass(i, 2 * pr, a0, b0);
      }
    if (np & 1) {  // the tile's last particle, alone
      const int p = np - 1;
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        cplx<double> a0[DIM];
        entries(i, p, a0);
        if (seg0 + i * NT < nseg) {
          SegWalk<double> w0(product(a0), step_phase(p));
#pragma unroll
          for (int j = 0; j < SEG; ++j) {
            acc[i][j].x += w0.cur.x;
            acc[i][j].y += w0.cur.y;
            if (j + 1 < SEG) w0.step(j);
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// launch helpers

inline int spt_for(int n_seg) {
  const int need = (n_seg + BLOCK - 1) / BLOCK;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 8;
}

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

inline int last_launch() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : int(e);
}

// Kernels asking for more than 64 KiB of LDS must raise their limit first
// (gfx950 has 160 KiB per workgroup processor).
template <typename F>
int allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 65536) return 0;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  return e == hipSuccess ? 0 : int(e);
}

inline int even(int x) { return (x + 1) & ~1; }
inline size_t up16(size_t x) { return (x + 15) & ~size_t(15); }

constexpr size_t RUN_LDS_BUDGET = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int RUN_NO_FIT = -1;                 // the fused kernel's LDS does not fit: use the per-step kernels

// Workgroups of this kernel that fit on one CU by registers (4 SIMDs, 512
// VGPRs per lane each); the fused kernel sizes its LDS so as not to lower it.
template <typename F>
int blocks_per_cu(F* kernel, int nt) {
  hipFuncAttributes a{};
  if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(kernel)) != hipSuccess || a.numRegs <= 0) return 1;
  const int vgpr = (a.numRegs + 7) & ~7;
  const int waves_per_simd = std::min(8, 512 / vgpr);
  return std::max(1, 4 * waves_per_simd / (nt / 64));
}

}  // namespace ewald
