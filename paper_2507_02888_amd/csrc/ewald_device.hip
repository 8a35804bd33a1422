// HIP kernels of libewald for gfx950 (MI355X).
//
// Mathematics: periodic Ewald energy and single-particle move deltas of the
// paper's Sec. 2.2 (Eqs. (2)-(6)); the plane-wave Jastrow value of Sec. 2.3
// (Eq. (9)) through the same structure factor; the separable phase identity
// of Eq. (10): exp(i G.r) = prod_d exp(2 pi i n_d s_d) for G = sum_d n_d b_d
// and fractional coordinates s = r A^-1.
//
// Layout (see ewald_internal.h): the half set of G vectors is stored as
// segments of SEG = 4 slots that are consecutive along the last reduced index.
// A segment's first phase is a product of per-dimension table entries and the
// following three are obtained by multiplying with exp(2 pi i s_last), one
// complex multiply per slot.  Slots are slot-planar (slot j of segment s at
// j * n_seg + s) so that one wave instruction reads 64 consecutive entries.
//
// One workgroup of 256 threads (four wave64s) serves one walker in every
// kernel; reductions are wave shuffles followed by a 4-entry LDS combine.
// Nothing here is a dense contraction worth an MFMA: the phase work is
// complex multiplies with K = 1 and the pair work is transcendental-bound.

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
  if (DIM == 3) {
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
    double ir[NE], t[NE], p[NE];
    const double scale = K.scale;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      ir[e] = rsqrt_pos(r2[e]);
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
    float t[NE], p[NE];
    double ir[NE];
    const float scale = float(K.scale);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      ir[e] = rsqrt_pos(r2[e]);
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

// Real-space part of a move of particle k from so to sn, summed over the
// mobile particles j != k (positions pos, charges q) and the fixed ions:
// sum_j q_j [phi(sn - s_j) - phi(so - s_j)].  Threads take j = tid, tid + NT, ...
// PPR particles (2 PPR pair terms) per round: 2 for workgroups of up to 512
// threads, 1 for 1024 (one particle per thread at N = 1024).  Indices are
// clamped rather than branched on, so every load is in bounds and the loop
// body has no divergent control flow.
template <int DIM, bool MIXED, int PD, int NT>
__device__ __forceinline__ double real_move(const double* sn, const double* so, int k, const double* pos,
                                            const double* q, int n, const DevSys* __restrict__ S) {
  constexpr int PPR = NT >= 1024 ? 1 : 2;
  const FrameK K = frame_k(S);
  PairAcc<MIXED, PD> pr(S->p64, S->p32, K);
  const int n_cand = S->n_cand;
  const double rc2 = S->rc2;
  for (int j0 = threadIdx.x; j0 < n; j0 += PPR * NT) {
    double qq[2 * PPR], r2[2 * PPR];
#pragma unroll
    for (int c = 0; c < PPR; ++c) {
      const int j = j0 + c * NT;
      const bool ok = j < n && j != k;
      const int jj = j < n ? j : n - 1;
      double sj[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) sj[d] = pos[jj * DIM + d];
      const double qj = ok ? q[jj] : 0.0;
      r2[2 * c] = ok ? min_r2<DIM>(sn, sj, S, n_cand) : rc2;
      r2[2 * c + 1] = ok ? min_r2<DIM>(so, sj, S, n_cand) : rc2;
      qq[2 * c] = qj;
      qq[2 * c + 1] = -qj;
    }
    pr.template add<2 * PPR>(qq, r2);
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
template <int DIM, bool MIXED, int PD, int NT, int PPR, bool ORTHO, bool XTRA>
__device__ __forceinline__ double real_move_own(const double* sn, const double* so, int k,
                                                const double (&ps)[PPR][DIM], const double (&pq)[PPR],
                                                const double* lpos, const double* lq, int n,
                                                const DevSys* __restrict__ S, const double* c64,
                                                const float* c32, const FrameK& K) {
  PairAcc<MIXED, PD> pr(c64, c32, K);
  const int n_cand = S->n_cand;
  const double rc2 = S->rc2;
  {
    double qq[2 * PPR], r2[2 * PPR];
#pragma unroll
    for (int c = 0; c < PPR; ++c) {
      const int j = threadIdx.x + c * NT;
      const bool ok = j < n && j != k;
      r2[2 * c] = ok ? image_r2<DIM, ORTHO>(sn, ps[c], S, n_cand, K) : rc2;
      r2[2 * c + 1] = ok ? image_r2<DIM, ORTHO>(so, ps[c], S, n_cand, K) : rc2;
      qq[2 * c] = pq[c];
      qq[2 * c + 1] = -pq[c];
    }
    pr.template add<2 * PPR>(qq, r2);
  }
  if (!XTRA) return pr.value();
  for (int j = threadIdx.x + PPR * NT; j < n; j += NT) {
    double qq[2], r2[2];
    const bool ok = j != k;
    double xj[DIM];
    geo_pos<DIM, ORTHO>(lpos + j * DIM, S, xj);
    r2[0] = ok ? image_r2<DIM, ORTHO>(sn, xj, S, n_cand, K) : rc2;
    r2[1] = ok ? image_r2<DIM, ORTHO>(so, xj, S, n_cand, K) : rc2;
    qq[0] = lq[j];
    qq[1] = -lq[j];
    pr.template add<2>(qq, r2);
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
template <int DIM, int NS, int NT = BLOCK>
__device__ void rebuild_rho(cplx<double> (&acc)[NS][SEG], const uint32_t (&an)[NS], int seg0,
                            const DevSys* __restrict__ S, const double* pos, const double* q, int n,
                            cplx<double>* tabs, int tile = TILE_P) {
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
        const double* rf = S->rho_fix + 2 * (size_t(j) * nseg + s);
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
// Energy: wrap positions, rho in FP64, reciprocal and Jastrow sums, real-space
// pairs, constants.  SPT = segments per thread held in registers.  Both
// precision forms compute the energy alike, in FP64: it adds ~N^2/4 pair terms
// of one sign (like charges), so any FP32 rounding bias of the pair function
// would add up coherently, while in a move delta it cancels between the old
// and new terms.  The pair loop works in the orthogonal-sublattice frame when
// the cell has one (ORTHO); rho is built from the fractional positions just
// stored in the walker state.
template <int DIM, int SPT, int PD, bool ORTHO>
__global__ __launch_bounds__(BLOCK, 4) void k_energy(const DevSys* __restrict__ systems,
                                                  const DevWalker* __restrict__ walkers,
                                                  const double* __restrict__ pos, char* __restrict__ state,
                                                  double* __restrict__ energy, double* __restrict__ jastrow,
                                                  int lds_pos, int tile) {
  extern __shared__ double smem[];
  const DevWalker W = walkers[blockIdx.x];
  const int w = W.id, tid = threadIdx.x;
  const DevSys* __restrict__ S = systems + W.sys;
  const int n = W.n_mobile, nseg = S->n_seg, nfix = S->n_fixed, n_cand = S->n_cand;
  char* st = state + W.state_off;
  WalkerHdr* hdr = reinterpret_cast<WalkerHdr*>(st);
  double* spos = reinterpret_cast<double*>(st + HDR_BYTES);
  double* rho = reinterpret_cast<double*>(st + HDR_BYTES + walker_pos_bytes(n, DIM));
  // LDS: the rebuild's phase-table tiles first, then (in the same space) the
  // pair loop's positions and charges
  double* red = smem;                        // [4 * 4]
  cplx<double>* tabs = reinterpret_cast<cplx<double>*>(smem + 16);
  double* lpos = smem + 16;                  // [n][DIM] in the pair loop's geometry
  double* lq = lpos + lds_pos * DIM;         // [n]

  const double* pw = pos + size_t(W.pos_off) * DIM;
  for (int i = tid; i < n; i += BLOCK) {
    double r[DIM], s[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) r[d] = pw[i * DIM + d];
    to_frac<DIM>(r, S->Ainv, s);
#pragma unroll
    for (int d = 0; d < DIM; ++d) spos[i * DIM + d] = s[d];
  }
  if (tid == 0) {
    hdr->counter = 0;
    hdr->pending_k = -1;
    hdr->n_accepts = 0;
    hdr->n_refresh = 0;
    hdr->pending_s[0] = hdr->pending_s[1] = hdr->pending_s[2] = 0.0;
    hdr->drift_max = 0.0;
  }
  __syncthreads();

  // reciprocal space
  uint32_t an[SPT];
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    const int s = tid + i * BLOCK;
    an[i] = s < nseg ? S->seg_n[s] : 0u;
  }
  cplx<double> acc[SPT][SEG];
  rebuild_rho<DIM, SPT>(acc, an, tid, S, spos, S->mobile_q, n, tabs, tile);
  double er = 0.0, ej = 0.0;
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    const int s = tid + i * BLOCK;
    if (s < nseg) {
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const size_t g = size_t(j) * nseg + s;
        const double m2 = acc[i][j].x * acc[i][j].x + acc[i][j].y * acc[i][j].y;
        er = fma(S->w[g], m2, er);
        if (S->ja) ej = fma(S->ja[g], m2, ej);
        rho[2 * g] = acc[i][j].x;
        rho[2 * g + 1] = acc[i][j].y;
      }
    }
  }

  // real space: each unordered mobile pair once (pair i with i+1..i+(n-1)/2
  // cyclically, plus i+n/2 for i < n/2 when n is even), then every fixed ion
  // positions in the pair loop's geometry replace the tiles (the rebuild
  // ends with a barrier)
  for (int i = tid; i < n; i += BLOCK) {
    double sv[DIM], x[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) sv[d] = spos[i * DIM + d];
    geo_pos<DIM, ORTHO>(sv, S, x);
#pragma unroll
    for (int d = 0; d < DIM; ++d) lpos[i * DIM + d] = x[d];
    lq[i] = S->mobile_q[i];
  }
  __syncthreads();
  // the pair loop's constants in vector registers (see frame_k_vector)
  const FrameK K = frame_k_vector(S);
  double cf64[PD + 1];
  {
    int z = 0;
    asm volatile("" : "+v"(z));
#pragma unroll
    for (int i = 0; i <= PD; ++i) cf64[i] = S->p64[i + z];
  }
  PairAcc<false, PD> pr(cf64, S->p32, K);
  const double rc2 = S->rc2;
  const int half = (n - 1) / 2;
  for (int i = tid; i < n; i += BLOCK) {
    double si[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) si[d] = lpos[i * DIM + d];
    const double qi = lq[i];
    const int n_mob = half + (((n & 1) == 0 && i < n / 2) ? 1 : 0);
    const int n_part = n_mob + nfix;
    for (int m0 = 0; m0 < n_part; m0 += 4) {
      double qq[4], r2[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int m = m0 + c;
        const bool mob = m < n_mob, fix = !mob && m < n_part;
        int j = i + m + 1;
        if (j >= n) j -= n;
        double sj[DIM];
        if (mob) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) sj[d] = lpos[j * DIM + d];
        } else {
          geo_pos<DIM, ORTHO>(S->fixed_s + (fix ? m - n_mob : 0) * DIM, S, sj);
        }
        qq[c] = mob ? qi * lq[j] : fix ? qi * S->fixed_q[m - n_mob] : 0.0;
        r2[c] = (mob || fix) ? image_r2<DIM, ORTHO>(si, sj, S, n_cand, K) : rc2;
      }
      pr.template add<4>(qq, r2);
    }
  }
  double v[3] = {pr.value(), er, ej};
  block_sum<3>(v, red);
  if (tid == 0) {
    energy[w] = v[0] + v[1] + S->e_const;
    if (jastrow) jastrow[w] = v[2];
  }
}

// ---------------------------------------------------------------------------
// Move delta: dE and dJ of moving particle k to new_pos; records the pending
// move.  rho is streamed from the state once (slot-planar, coalesced).
template <int DIM, bool MIXED, int PD>
__global__ __launch_bounds__(BLOCK, 4) void k_delta(const DevSys* __restrict__ systems,
                                                 const DevWalker* __restrict__ walkers, char* __restrict__ state,
                                                 const int32_t* __restrict__ kk, const double* __restrict__ new_pos,
                                                 double* __restrict__ delta, double* __restrict__ djas, int lds_tab) {
  using R = typename std::conditional<MIXED, float, double>::type;
  using WT2 = cplx<R>;  // (weight, Jastrow coefficient) in the form's precision
  extern __shared__ double smem[];
  const DevWalker W = walkers[blockIdx.x];
  const int w = W.id, tid = threadIdx.x;
  const DevSys* __restrict__ S = systems + W.sys;
  const int n = W.n_mobile, nseg = S->n_seg, nm = S->nm;
  const int tbl = 2 * nm + 1;
  char* st = state + W.state_off;
  WalkerHdr* hdr = reinterpret_cast<WalkerHdr*>(st);
  const double* spos = reinterpret_cast<const double*>(st + HDR_BYTES);
  const double* rho = reinterpret_cast<const double*>(st + HDR_BYTES + walker_pos_bytes(n, DIM));
  double* red = smem;
  cplx<R>* to = reinterpret_cast<cplx<R>*>(smem + 16);
  cplx<R>* tn = to + DIM * tbl;
  WT2* ltab = reinterpret_cast<WT2*>(smem + 16 + lds_tab);  // shell table (when it fits)
  const double2* __restrict__ rho2 = reinterpret_cast<const double2*>(rho);

  const int k = kk[w];
  if (k < 0 || k >= n) {
    if (tid == 0) {
      delta[w] = NAN;
      if (djas) djas[w] = NAN;
      hdr->pending_k = -1;
    }
    return;
  }
  // start streaming this thread's first segment of rho before the table barrier
  const bool wlds = S->wtab_lds != 0;
  double2 rcur[SEG];
  uint32_t scur[SEG];
#pragma unroll
  for (int j = 0; j < SEG; ++j) {
    const size_t g = size_t(j) * nseg + (tid < nseg ? tid : 0);
    rcur[j] = rho2[g];
    scur[j] = S->slot_shell[g];
  }
  if (wlds)
    for (int i = tid; i < S->n_wtab; i += BLOCK) ltab[i] = {R(S->wa_tab[2 * i]), R(S->wa_tab[2 * i + 1])};
  double sn[DIM], so[DIM];
  {
    double r[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) r[d] = new_pos[size_t(w) * DIM + d];
    to_frac<DIM>(r, S->Ainv, sn);
#pragma unroll
    for (int d = 0; d < DIM; ++d) so[d] = spos[k * DIM + d];
  }
  const double qk = S->mobile_q[k];
  if (tid < 2 * DIM) fill_row<R>(to + tid * tbl, pick_coord<DIM>(so, sn, tid), nm);  // to, then tn
  __syncthreads();

  // reciprocal space: t(G) = 2 q Re(conj(rho) d) + q^2 |d|^2, d = e_new - e_old
  const cplx<R> uo = tab_at(to, DIM - 1, nm + 1, tbl), un = tab_at(tn, DIM - 1, nm + 1, tbl);
  const double* __restrict__ wt = S->w;
  const double* __restrict__ ja = S->ja;
  // t(G) = q^2 [dx (dx + (2/q) rho_x) + dy (dy + (2/q) rho_y)]: q^2 is applied
  // once to the sums, and a neutral particle's move changes nothing
  double accE64 = 0.0, accJ64 = 0.0;
  Kahan accE32, accJ32;
  const R c2q = qk != 0.0 ? R(2.0 / qk) : R(0);
  for (int s = tid; s < nseg && qk != 0.0; s += BLOCK) {
    // prefetch the next segment while this one is consumed
    const int s2 = s + BLOCK < nseg ? s + BLOCK : s;
    double2 rnxt[SEG];
    uint32_t snxt[SEG];
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const size_t g2 = size_t(j) * nseg + s2;
      rnxt[j] = rho2[g2];
      snxt[j] = S->slot_shell[g2];
    }
    const uint32_t pn = S->seg_n[s];
    SegWalk<R> wo(anchor<DIM, R>(to, pn, nm), uo), wn(anchor<DIM, R>(tn, pn, nm), un);
    float segE = 0.f, segJ = 0.f;  // mixed form: FP32 sums per segment, compensated across segments
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const cplx<R> eo = wo.cur, en = wn.cur;
      const size_t g = size_t(j) * nseg + s;
      R wg, aj;
      if (wlds) {
        const WT2 wa = ltab[scur[j]];
        wg = wa.x;
        aj = wa.y;
      } else {
        wg = R(wt[g]);
        aj = ja ? R(ja[g]) : R(0);
      }
      const R dx = en.x - eo.x, dy = en.y - eo.y;
      const R ux = fma(c2q, R(rcur[j].x), dx), uy = fma(c2q, R(rcur[j].y), dy);
      const R t = fma(ux, dx, uy * dy);
      if (MIXED) {
        segE = fmaf(float(wg), float(t), segE);
        if (ja) segJ = fmaf(float(aj), float(t), segJ);
      } else {
        accE64 = fma(double(wg), double(t), accE64);
        if (ja) accJ64 = fma(double(aj), double(t), accJ64);
      }
      if (j + 1 < SEG) {
        wo.step(j);
        wn.step(j);
      }
    }
    if (MIXED) {
      accE32.add(segE);
      if (ja) accJ32.add(segJ);
    }
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      rcur[j] = rnxt[j];
      scur[j] = snxt[j];
    }
  }
  // real space
  const double er = real_move<DIM, MIXED, PD, BLOCK>(sn, so, k, spos, S->mobile_q, n, S);
  const double q2 = qk * qk;
  double v[2] = {q2 * (MIXED ? accE32.value() : accE64) + qk * er, q2 * (MIXED ? accJ32.value() : accJ64)};
  block_sum<2>(v, red);
  if (tid == 0) {
    delta[w] = v[0];
    if (djas) djas[w] = v[1];
    hdr->pending_k = k;
#pragma unroll
    for (int d = 0; d < 3; ++d) hdr->pending_s[d] = d < DIM ? sn[d] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Accept / reject the pending move.  rho += q (e_new - e_old) with the
// difference formed in the form's precision and added in FP64.
template <int DIM, bool MIXED>
__global__ __launch_bounds__(BLOCK) void k_accept(const DevSys* __restrict__ systems,
                                                  const DevWalker* __restrict__ walkers, char* __restrict__ state,
                                                  const uint8_t* __restrict__ accept) {
  using R = typename std::conditional<MIXED, float, double>::type;
  extern __shared__ double smem[];
  const DevWalker W = walkers[blockIdx.x];
  const int w = W.id, tid = threadIdx.x;
  const DevSys* __restrict__ S = systems + W.sys;
  const int n = W.n_mobile, nseg = S->n_seg, nm = S->nm, K = S->refresh_every;
  const int tbl = 2 * nm + 1;
  char* st = state + W.state_off;
  WalkerHdr* hdr = reinterpret_cast<WalkerHdr*>(st);
  double* spos = reinterpret_cast<double*>(st + HDR_BYTES);
  double* rho = reinterpret_cast<double*>(st + HDR_BYTES + walker_pos_bytes(n, DIM));
  cplx<R>* to = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* tn = to + DIM * tbl;

  const int pk = hdr->pending_k;
  int counter = hdr->counter;
  const bool acc = pk >= 0 && pk < n && accept[w] != 0;
  double so[DIM], sn[DIM];
  if (acc) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      so[d] = spos[pk * DIM + d];
      sn[d] = hdr->pending_s[d];
    }
    if (tid < 2 * DIM) fill_row<R>(to + tid * tbl, pick_coord<DIM>(so, sn, tid), nm);  // to, then tn
  }
  __syncthreads();  // every thread has read the header and pending position
  if (acc) {
    const R q = R(S->mobile_q[pk]);
    const cplx<R> uo = tab_at(to, DIM - 1, nm + 1, tbl), un = tab_at(tn, DIM - 1, nm + 1, tbl);
    double2* rho2 = reinterpret_cast<double2*>(rho);
    for (int s = tid; s < nseg; s += BLOCK) {
      double2 r[SEG];
#pragma unroll
      for (int j = 0; j < SEG; ++j) r[j] = rho2[size_t(j) * nseg + s];
      const uint32_t pn = S->seg_n[s];
      SegWalk<R> wo(anchor<DIM, R>(to, pn, nm), uo), wn(anchor<DIM, R>(tn, pn, nm), un);
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        r[j].x += double(q * (wn.cur.x - wo.cur.x));
        r[j].y += double(q * (wn.cur.y - wo.cur.y));
        rho2[size_t(j) * nseg + s] = r[j];
        if (j + 1 < SEG) {
          wo.step(j);
          wn.step(j);
        }
      }
    }
  }
  if (tid == 0) {
    if (K > 0 && counter >= K) counter = 0;  // rho was rebuilt after the previous call
    if (acc) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) spos[pk * DIM + d] = sn[d];
      counter += 1;
      hdr->n_accepts += 1;
    }
    hdr->counter = counter;
    hdr->pending_k = -1;
  }
}

// Rebuild rho in FP64 for walkers whose accepted-move counter reached K.
// grid = (walkers, chunks); chunk c rebuilds segments [c*BLOCK, (c+1)*BLOCK).
// The counter is reset by the next accept or run call, not here, so that
// every chunk sees the same trigger.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_rebuild(const DevSys* __restrict__ systems,
                                                   const DevWalker* __restrict__ walkers,
                                                   char* __restrict__ state) {
  extern __shared__ double smem[];
  const DevWalker W = walkers[blockIdx.x];
  const int chunk = blockIdx.y, tid = threadIdx.x;
  const DevSys* __restrict__ S = systems + W.sys;
  const int n = W.n_mobile, nseg = S->n_seg, K = S->refresh_every;
  char* st = state + W.state_off;
  WalkerHdr* hdr = reinterpret_cast<WalkerHdr*>(st);
  if (K <= 0 || hdr->counter < K || chunk * BLOCK >= nseg) return;  // uniform per workgroup
  const double* spos = reinterpret_cast<const double*>(st + HDR_BYTES);
  double* rho = reinterpret_cast<double*>(st + HDR_BYTES + walker_pos_bytes(n, DIM));
  cplx<double>* tabs = reinterpret_cast<cplx<double>*>(smem);
  const int s = chunk * BLOCK + tid;
  uint32_t an[1] = {s < nseg ? S->seg_n[s] : 0u};
  cplx<double> acc[1][SEG];
  rebuild_rho<DIM, 1>(acc, an, chunk * BLOCK + tid, S, spos, S->mobile_q, n, tabs);
  if (s < nseg) {
    double drift = 0.0;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const size_t g = size_t(j) * nseg + s;
      drift = fmax(drift, fmax(fabs(acc[0][j].x - rho[2 * g]), fabs(acc[0][j].y - rho[2 * g + 1])));
      rho[2 * g] = acc[0][j].x;
      rho[2 * g + 1] = acc[0][j].y;
    }
    for (int off = 32; off > 0; off >>= 1) drift = fmax(drift, __shfl_xor(drift, off, 64));
    if ((tid & 63) == 0)
      atomicMax(reinterpret_cast<unsigned long long*>(&hdr->drift_max),
                static_cast<unsigned long long>(__double_as_longlong(drift)));
  }
  if (chunk == 0 && tid == 0) hdr->n_refresh += 1;
}

// ---------------------------------------------------------------------------
// Fused multi-move: n_steps proposals per walker with rho, the shell-table
// offsets, the segment anchors and the thread's own particles in registers,
// and positions, charges, the shell table and the chunk's phase tables in LDS
// for the whole sequence.  NT threads per walker, SPT segments per thread.
//
// Moves are processed in chunks of up to `ch` with no barrier inside a chunk.
// Every piece of cross-thread information a move needs is fixed before the
// chunk starts:
//   - the proposals are staged in LDS, together with each move's old
//     position (the latest accepted earlier move of the same particle in the
//     chunk, else the position at the chunk start);
//   - the per-dimension phase tables of every move's old and new position
//     are built by the whole workgroup, once per chunk;
//   - thread t owns the slots of its segments (it alone updates them) and the
//     particles j = t, t + NT, ... (it alone reads and updates them during
//     the chunk);
//   - each wave reduces its partial sums per row of 16 lanes with DPP and
//     parks the four row sums in LDS; the cross-row sums of the chunk are
//     formed after the chunk, in a fixed order.
// A chunk ends early after a move that brings the accept counter to K, so the
// FP64 rebuild of the mixed form runs between chunks.
struct RunLds {
  // byte offsets into dynamic LDS; positions start at 0
  uint32_t q, red, wtab, ctab, sn, so, xn, xo, c2q, part, k, acc, cnt;
  uint32_t rcopy;  // 0, or the LDS copy of the running rho during a rebuild
  int ch;     // moves per chunk
  int rtile;  // particles per rebuild tile (the tiles reuse the chunk tables)
};

// At least two waves per SIMD for workgroups of up to 512 threads (the
// register budget stays within 256 per lane; without the bound the compiler
// may take accumulation registers as well, which leaves one wave per SIMD).
template <int DIM, bool MIXED, int NT, int SPT, int PPR, bool JAS, int PD, bool ORTHO, bool XTRA>
__global__ __launch_bounds__(NT, NT >= 1024 ? 4 : 2) void k_run(const DevSys* __restrict__ systems,
                                            const DevWalker* __restrict__ walkers, char* __restrict__ state,
                                            int n_steps, int n_walkers, const int32_t* __restrict__ kk,
                                            const double* __restrict__ new_pos, const uint8_t* __restrict__ accept,
                                            double* __restrict__ delta, double* __restrict__ djas, RunLds L) {
  using R = typename std::conditional<MIXED, float, double>::type;
  using WT = R;          // the mixed form multiplies weights with FP32 terms
  using WT2 = cplx<WT>;  // (weight, Jastrow coefficient)
  constexpr int NW = NT / 64;
  // PPR: own particles per thread held in registers (particles j = t + c NT, c < PPR)
  extern __shared__ __align__(16) char lds[];
  const DevWalker W = walkers[blockIdx.x];
  const int w = W.id, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const DevSys* __restrict__ S = systems + W.sys;
  const int n = W.n_mobile, nseg = S->n_seg, nm = S->nm;
  const int K = S->refresh_every, tbl = 2 * nm + 1;
  const int mstride = 2 * DIM * tbl;  // one move's tables (old, new), in entries
  const int CH = L.ch;
  char* st = state + W.state_off;
  WalkerHdr* hdr = reinterpret_cast<WalkerHdr*>(st);
  double* spos = reinterpret_cast<double*>(st + HDR_BYTES);
  double* rho = reinterpret_cast<double*>(st + HDR_BYTES + walker_pos_bytes(n, DIM));
  double* lpos = reinterpret_cast<double*>(lds);
  double* lq = reinterpret_cast<double*>(lds + L.q);
  double* red = reinterpret_cast<double*>(lds + L.red);
  WT2* ltab = reinterpret_cast<WT2*>(lds + L.wtab);
  cplx<R>* ctab = reinterpret_cast<cplx<R>*>(lds + L.ctab);
  cplx<double>* tabs = reinterpret_cast<cplx<double>*>(lds + L.ctab);  // rebuild tiles, between chunks
  double* st_sn = reinterpret_cast<double*>(lds + L.sn);
  double* st_so = reinterpret_cast<double*>(lds + L.so);
  double* st_xn = reinterpret_cast<double*>(lds + L.xn);  // sn, so in the real-space geometry (ORTHO)
  double* st_xo = reinterpret_cast<double*>(lds + L.xo);
  double* st_c2q = reinterpret_cast<double*>(lds + L.c2q);  // 2 / q_k of each move (0 for q_k = 0)
  double* st_part = reinterpret_cast<double*>(lds + L.part);  // [CH][NW][4 rows][2]
  int* st_k = reinterpret_cast<int*>(lds + L.k);
  int* st_acc = reinterpret_cast<int*>(lds + L.acc);
  int* st_cnt = reinterpret_cast<int*>(lds + L.cnt);

  for (int i = tid; i < n * DIM; i += NT) lpos[i] = spos[i];
  for (int i = tid; i < n; i += NT) lq[i] = S->mobile_q[i];
  // every system of the batch has its shell table in LDS (checked by the launcher)
  for (int i = tid; i < S->n_wtab; i += NT) ltab[i] = {WT(S->wa_tab[2 * i]), WT(S->wa_tab[2 * i + 1])};
  int counter = hdr->counter;
  int n_acc = hdr->n_accepts, n_ref = hdr->n_refresh;
  double drift = hdr->drift_max;
  if (K > 0 && counter >= K) counter = 0;

  double ps[PPR][DIM], pq[PPR];
#pragma unroll
  for (int c = 0; c < PPR; ++c) {
    const int j = tid + c * NT;
    double sj[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) sj[d] = j < n ? spos[j * DIM + d] : 0.0;
    geo_pos<DIM, ORTHO>(sj, S, ps[c]);
    pq[c] = j < n ? S->mobile_q[j] : 0.0;
  }
  // Workgroups of up to 512 threads (256 vector registers per lane) hold the
  // pair-polynomial coefficients in vector registers for the whole sweep
  // (loaded with a lane-varying index, so they are not taken for scalars);
  // that leaves the scalar registers to the loop state, which otherwise
  // spills into vector-register lanes.  With 1024 threads they stay scalar.
  constexpr int PF = PD == 16 ? 12 : 22;
  constexpr bool CV = NT <= 512;
  double cf64[CV ? PD + 1 : 1];
  float cf32[CV ? PF + 1 : 1];
  if (CV) {
    int z = 0;
    asm volatile("" : "+v"(z));
#pragma unroll
    for (int i = 0; i <= (CV ? PD : 0); ++i) cf64[i] = S->p64[i + z];
#pragma unroll
    for (int i = 0; i <= (CV ? PF : 0); ++i) cf32[i] = S->p32[i + z];
  }
  const double* c64 = CV ? cf64 : S->p64;
  const float* c32 = CV ? cf32 : S->p32;
  FrameK fk{};  // with 1024 threads the constants are read where they are used
  if (CV) fk = frame_k_vector(S);
  uint32_t an[SPT];
  cplx<double> rv[SPT][SEG];
  uint32_t shp[SPT][SEG / 2];  // two 16-bit shell-table byte offsets per register
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    const int s = tid + i * NT;
    an[i] = s < nseg ? S->seg_n[s] : 0u;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const size_t g = size_t(j) * nseg + s;
      rv[i][j] = s < nseg ? cplx<double>{rho[2 * g], rho[2 * g + 1]} : cplx<double>{0.0, 0.0};
    }
#pragma unroll
    for (int j = 0; j < SEG; j += 2) {
      const size_t g = size_t(j) * nseg + s;
      shp[i][j / 2] = s < nseg ? uint32_t(S->slot_shell[g]) * uint32_t(sizeof(WT2)) |
                                     (uint32_t(S->slot_shell[g + nseg]) * uint32_t(sizeof(WT2)) << 16)
                               : 0u;
    }
  }
  __syncthreads();

  for (int m0 = 0; m0 < n_steps;) {
    // ---- stage the chunk: proposals, old positions, accept counts ----
    const int cnt = min(CH, n_steps - m0);
    if (tid < cnt) {
      const size_t idx = size_t(m0 + tid) * n_walkers + w;
      const int kv = kk[idx];
      st_k[tid] = (kv < 0 || kv >= n) ? -1 : kv;
      st_acc[tid] = accept[idx] != 0;
      double r[DIM], sv[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) r[d] = new_pos[idx * DIM + d];
      to_frac<DIM>(r, S->Ainv, sv);
#pragma unroll
      for (int d = 0; d < DIM; ++d) st_sn[tid * DIM + d] = sv[d];
    }
    __syncthreads();
    if (tid < cnt) {
      const int k = st_k[tid];
      int prev = -1, c = counter;
      for (int q = 0; q < tid; ++q) {
        const bool a = st_k[q] >= 0 && st_acc[q] != 0;
        if (a && st_k[q] == k) prev = q;
        c += a ? 1 : 0;
      }
      if (k >= 0) {
        double so[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          so[d] = prev >= 0 ? st_sn[prev * DIM + d] : lpos[k * DIM + d];
          st_so[tid * DIM + d] = so[d];
        }
        if (ORTHO) {
          frame_coords<DIM>(so, S, st_xo + tid * DIM);
          frame_coords<DIM>(st_sn + tid * DIM, S, st_xn + tid * DIM);
        }
        st_c2q[tid] = lq[k] != 0.0 ? 2.0 / lq[k] : 0.0;
      }
      st_cnt[tid] = c + ((k >= 0 && st_acc[tid] != 0) ? 1 : 0);  // accepts since the rebuild, after this move
    }
    __syncthreads();
    int len = cnt;
    if (MIXED && K > 0)
      for (int q = 0; q < cnt; ++q)
        if (st_cnt[q] >= K) {
          len = q + 1;
          break;
        }
    // ---- phase tables of every move of the chunk (old, then new position) ----
    // row e: move e / (2 DIM), old (0) or new (1) position, dimension; the
    // tables of a move are [old: DIM rows][new: DIM rows]
    for (int e = tid; e < len * 2 * DIM; e += NT) {
      const int q = e / (2 * DIM), r = e - q * (2 * DIM);
      if (st_k[q] >= 0)
        fill_row<R>(ctab + e * tbl, r < DIM ? st_so[q * DIM + r] : st_sn[q * DIM + r - DIM], nm);
    }
    __syncthreads();

    // ---- the chunk's moves, no barrier ----
    for (int mm = 0; mm < len; ++mm) {
      const int k = st_k[mm];
      double v0 = 0.0, v1 = 0.0;
      if (k >= 0) {  // uniform
        const bool acc = st_acc[mm] != 0;
        const double qk = lq[k];
        double sn[DIM], xn[DIM], xo[DIM];  // new (fractional), new and old in the real-space geometry
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          sn[d] = st_sn[mm * DIM + d];
          xn[d] = ORTHO ? st_xn[mm * DIM + d] : sn[d];
          xo[d] = ORTHO ? st_xo[mm * DIM + d] : st_so[mm * DIM + d];
        }
        if (qk != 0.0) {  // uniform; a neutral particle's move changes nothing
          const cplx<R>* to = ctab + mm * mstride;
          const cplx<R>* tn = to + DIM * tbl;
          const cplx<R> uo = tab_at(to, DIM - 1, nm + 1, tbl), un = tab_at(tn, DIM - 1, nm + 1, tbl);
          // t(G) = q^2 [dx (dx + (2/q) rho_x) + dy (dy + (2/q) rho_y)], q^2 applied to the sums
          const R q = R(qk), c2q = R(st_c2q[mm]);
          double accE64 = 0.0, accJ64 = 0.0;
          Kahan accE32, accJ32;  // mixed form: FP32 sums per segment, compensated across segments
#pragma unroll
          for (int i = 0; i < SPT; ++i) {
            if (tid + i * NT < nseg) {
              SegWalk<R> wo(anchor<DIM, R>(to, an[i], nm), uo), wn(anchor<DIM, R>(tn, an[i], nm), un);
              float segE = 0.f, segJ = 0.f;
#pragma unroll
              for (int j = 0; j < SEG; ++j) {
                const cplx<R> eo = wo.cur, en = wn.cur;
                const WT2 wa = ld_at_byte(ltab, (shp[i][j >> 1] >> (16 * (j & 1))) & 0xffffu);
                const R dx = en.x - eo.x, dy = en.y - eo.y;
                const R ux = fma(c2q, R(rv[i][j].x), dx), uy = fma(c2q, R(rv[i][j].y), dy);
                const R t = fma(ux, dx, uy * dy);
                if (MIXED) {
                  segE = fmaf(float(wa.x), float(t), segE);
                  if (JAS) segJ = fmaf(float(wa.y), float(t), segJ);
                } else {
                  accE64 = fma(double(wa.x), double(t), accE64);
                  if (JAS) accJ64 = fma(double(wa.y), double(t), accJ64);
                }
                if (acc) {
                  rv[i][j].x += double(q * dx);
                  rv[i][j].y += double(q * dy);
                }
                if (j + 1 < SEG) {
                  wo.step(j);
                  wn.step(j);
                }
              }
              if (MIXED) {
                accE32.add(segE);
                if (JAS) accJ32.add(segJ);
              }
            }
          }
          const double q2 = qk * qk;
          v0 = q2 * (MIXED ? accE32.value() : accE64);
          if (JAS) v1 = q2 * (MIXED ? accJ32.value() : accJ64);
          v0 += qk * real_move_own<DIM, MIXED, PD, NT, PPR, ORTHO, XTRA>(xn, xo, k, ps, pq, lpos, lq, n, S, c64, c32,
                                                                CV ? fk : frame_k(S));
        }
        if (acc) {
          if ((k % NT) == tid) {  // the owner moves its particle
#pragma unroll
            for (int d = 0; d < DIM; ++d) lpos[k * DIM + d] = sn[d];
#pragma unroll
            for (int c = 0; c < PPR; ++c)
              if (k == tid + c * NT)
#pragma unroll
                for (int d = 0; d < DIM; ++d) ps[c][d] = xn[d];
          }
          n_acc += 1;
        }
      }
      v0 = row_sum16(v0);
      if (JAS) v1 = row_sum16(v1);
      if ((lane & 15) == 0) {
        double* p = st_part + ((mm * NW + wave) * 4 + (lane >> 4)) * 2;
        p[0] = v0;
        p[1] = v1;
      }
    }
    if (len > 0) counter = st_cnt[len - 1];
    __syncthreads();  // partials and owner position updates complete

    // ---- outputs of the chunk (cross-row sums in a fixed order) ----
    if (tid < len) {
      const size_t idx = size_t(m0 + tid) * n_walkers + w;
      double e = 0.0, j = 0.0;
      if (st_k[tid] < 0) {
        e = j = NAN;
      } else {
        const double* p = st_part + tid * NW * 8;
#pragma unroll
        for (int v = 0; v < NW * 4; ++v) {
          e += p[2 * v];
          j += p[2 * v + 1];
        }
      }
      delta[idx] = e;
      if (djas) djas[idx] = j;
    }
    if (MIXED && K > 0 && counter >= K) {  // uniform: rebuild rho in FP64 between chunks
      __syncthreads();  // the chunk's outputs have been read from the staging area
      // keep the running rho for the drift check: in LDS when the layout has
      // room for it, else in the walker state
      cplx<double>* rc = reinterpret_cast<cplx<double>*>(lds + L.rcopy);
#pragma unroll
      for (int i = 0; i < SPT; ++i) {
        const int s = tid + i * NT;
        if (s < nseg)
#pragma unroll
          for (int j = 0; j < SEG; ++j) {
            if (L.rcopy) {
              rc[(i * NT + tid) * SEG + j] = rv[i][j];
            } else {
              const size_t g = size_t(j) * nseg + s;
              rho[2 * g] = rv[i][j].x;
              rho[2 * g + 1] = rv[i][j].y;
            }
          }
      }
      rebuild_rho<DIM, SPT, NT>(rv, an, tid, S, lpos, lq, n, tabs, L.rtile);
      double dm = 0.0;
#pragma unroll
      for (int i = 0; i < SPT; ++i) {
        const int s = tid + i * NT;
        if (s < nseg)
#pragma unroll
          for (int j = 0; j < SEG; ++j) {
            cplx<double> old;
            if (L.rcopy) {
              old = rc[(i * NT + tid) * SEG + j];
            } else {
              const size_t g = size_t(j) * nseg + s;
              old = {rho[2 * g], rho[2 * g + 1]};
            }
            dm = fmax(dm, fmax(fabs(rv[i][j].x - old.x), fabs(rv[i][j].y - old.y)));
          }
      }
      for (int off = 32; off > 0; off >>= 1) dm = fmax(dm, __shfl_xor(dm, off, 64));
      if (lane == 0) red[wave] = dm;
      __syncthreads();
      for (int k2 = 0; k2 < NW; ++k2) drift = fmax(drift, red[k2]);
      counter = 0;
      n_ref += 1;
    }
    __syncthreads();  // staging buffers and tables are reused by the next chunk
    m0 += len;
  }

  // write back (n_acc counted by every thread alike)
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    const int s = tid + i * NT;
    if (s < nseg)
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const size_t g = size_t(j) * nseg + s;
        rho[2 * g] = rv[i][j].x;
        rho[2 * g + 1] = rv[i][j].y;
      }
  }
  for (int i = tid; i < n * DIM; i += NT) spos[i] = lpos[i];
  if (tid == 0) {
    hdr->counter = counter;
    hdr->n_accepts = n_acc;
    hdr->n_refresh = n_ref;
    hdr->pending_k = -1;
    hdr->drift_max = drift;
  }
}

// ---------------------------------------------------------------------------
// launchers

namespace {

int spt_for(int n_seg) {
  const int need = (n_seg + BLOCK - 1) / BLOCK;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 8;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

int last_launch() {
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

int even(int x) { return (x + 1) & ~1; }

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


template <int DIM, int SPT, int PD, bool ORTHO>
int energy_inst(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
                void* stream) {
  const int lds_pos = even(b.max_particles);
  const size_t rpart = size_t(DIM) * (2 * b.max_nm + 1) * sizeof(cplx<double>);
  const size_t head = 16 * 8, pairs = size_t(lds_pos) * (DIM + 1) * 8;
  auto* kern = k_energy<DIM, SPT, PD, ORTHO>;
  // rebuild tiles (sharing their LDS with the pair loop's positions) as
  // large as LDS allows without lowering the workgroups per CU that
  // registers allow (four: the kernel is bounded to four waves per SIMD),
  // at most 64
  static const int per_cu = blocks_per_cu(kern, BLOCK);
  const size_t budget = RUN_LDS_BUDGET / size_t(per_cu);
  int tile = budget > head ? int(std::min<size_t>((budget - head) / rpart, 64)) : 0;
  tile = std::max(tile & ~1, TILE_P);  // even (the tiles interleave particle pairs)
  const size_t lds = head + std::max(pairs, size_t(tile) * rpart);
  if (int rc = allow_lds(kern, lds)) return rc;
  hipLaunchKernelGGL(kern, dim3(b.n_walkers), dim3(BLOCK), lds, as_stream(stream), b.d_sys, b.d_walk, pos, state,
                     energy, jastrow, lds_pos, tile);
  return last_launch();
}

template <int DIM, int PD, bool ORTHO>
int energy_pd(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
              void* stream) {
  switch (spt_for(b.max_n_seg)) {
    case 1: return energy_inst<DIM, 1, PD, ORTHO>(b, pos, state, energy, jastrow, stream);
    case 2: return energy_inst<DIM, 2, PD, ORTHO>(b, pos, state, energy, jastrow, stream);
    case 4: return energy_inst<DIM, 4, PD, ORTHO>(b, pos, state, energy, jastrow, stream);
    default: return energy_inst<DIM, 8, PD, ORTHO>(b, pos, state, energy, jastrow, stream);
  }
}

template <int DIM>
int energy_dim(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
               void* stream) {
  const bool o = b.all_ortho && !b.general_frame;
  if (b.poly_deg <= 16)
    return o ? energy_pd<DIM, 16, true>(b, pos, state, energy, jastrow, stream)
             : energy_pd<DIM, 16, false>(b, pos, state, energy, jastrow, stream);
  return o ? energy_pd<DIM, 32, true>(b, pos, state, energy, jastrow, stream)
           : energy_pd<DIM, 32, false>(b, pos, state, energy, jastrow, stream);
}

template <int DIM, bool MIXED>
int delta_dim(const LaunchBatch& b, char* state, const int32_t* k, const double* new_pos, double* delta,
              double* djas, void* stream) {
  using R = typename std::conditional<MIXED, float, double>::type;
  const size_t mtab = size_t(2) * DIM * (2 * b.max_nm + 1) * sizeof(cplx<R>);
  const int lds_tab = even(int((mtab + 7) / 8));  // in doubles
  const size_t lds = 16 * 8 + size_t(lds_tab) * 8 + size_t(b.max_wtab) * sizeof(cplx<R>);
  if (b.poly_deg <= 16)
    hipLaunchKernelGGL((k_delta<DIM, MIXED, 16>), dim3(b.n_walkers), dim3(BLOCK), lds, as_stream(stream),
                       b.d_sys, b.d_walk, state, k, new_pos, delta, djas, lds_tab);
  else
    hipLaunchKernelGGL((k_delta<DIM, MIXED, 32>), dim3(b.n_walkers), dim3(BLOCK), lds, as_stream(stream),
                       b.d_sys, b.d_walk, state, k, new_pos, delta, djas, lds_tab);
  return last_launch();
}

template <int DIM, bool MIXED>
int accept_dim(const LaunchBatch& b, char* state, const uint8_t* accept, void* stream) {
  using R = typename std::conditional<MIXED, float, double>::type;
  const size_t lds = size_t(2) * DIM * (2 * b.max_nm + 1) * sizeof(cplx<R>);
  hipLaunchKernelGGL((k_accept<DIM, MIXED>), dim3(b.n_walkers), dim3(BLOCK), lds, as_stream(stream), b.d_sys,
                     b.d_walk, state, accept);
  int rc = last_launch();
  if (rc || !MIXED || b.refresh_every <= 0) return rc;
  const size_t lds_r = size_t(TILE_P) * DIM * (2 * b.max_nm + 1) * sizeof(cplx<double>);
  const int chunks = (b.max_n_seg + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL((k_rebuild<DIM>), dim3(b.n_walkers, chunks), dim3(BLOCK), lds_r, as_stream(stream), b.d_sys,
                     b.d_walk, state);
  return last_launch();
}


size_t up16(size_t x) { return (x + 15) & ~size_t(15); }

// LDS layout of the fused kernel for a chunk of ch moves; returns the total bytes.
template <int DIM, bool MIXED, int NT, int SPT>
size_t run_layout(const LaunchBatch& b, int ch, RunLds& L) {
  using R = typename std::conditional<MIXED, float, double>::type;
  constexpr int NW = NT / 64;
  const size_t tbl = size_t(2 * b.max_nm + 1);
  const size_t mtab = 2 * DIM * tbl * sizeof(cplx<R>);                 // one move's tables
  const size_t rpart = DIM * tbl * sizeof(cplx<double>);               // one rebuild particle
  size_t o = up16(size_t(b.max_particles) * DIM * 8);
  L.q = uint32_t(o);
  o = up16(o + size_t(b.max_particles) * 8);
  L.red = uint32_t(o);
  o = up16(o + size_t(NW) * 8);
  L.wtab = uint32_t(o);
  o = up16(o + size_t(b.max_wtab) * sizeof(cplx<R>));
  L.ctab = uint32_t(o);
  const size_t ctab = std::max(size_t(ch) * mtab, size_t(TILE_P) * rpart);
  o = up16(o + ctab);
  L.sn = uint32_t(o);
  o = up16(o + size_t(ch) * DIM * 8);
  L.so = uint32_t(o);
  o = up16(o + size_t(ch) * DIM * 8);
  L.xn = uint32_t(o);
  o = up16(o + size_t(ch) * DIM * 8);
  L.xo = uint32_t(o);
  o = up16(o + size_t(ch) * DIM * 8);
  L.c2q = uint32_t(o);
  o = up16(o + size_t(ch) * 8);
  L.part = uint32_t(o);
  o = up16(o + size_t(ch) * NW * 8 * 8);
  L.k = uint32_t(o);
  o = up16(o + size_t(ch) * 4);
  L.acc = uint32_t(o);
  o = up16(o + size_t(ch) * 4);
  L.cnt = uint32_t(o);
  o = up16(o + size_t(ch) * 4);
  L.ch = ch;
  L.rtile = int(std::min<size_t>(ctab / rpart, 64)) & ~1;  // even (the tiles interleave particle pairs)
  // Between chunks the tables and the staging area are free: the mixed form's
  // rebuild keeps the running rho there (for the drift check) when it fits
  // beside tiles of at least TILE_P particles, instead of a round trip
  // through HBM.
  L.rcopy = 0;
  const size_t rcopy = size_t(SPT) * NT * SEG * sizeof(cplx<double>);
  const size_t region = o - L.ctab;
  if (MIXED && region >= rcopy + size_t(TILE_P) * rpart) {
    L.rcopy = uint32_t((o - rcopy) & ~size_t(15));
    L.rtile = int(std::min<size_t>((L.rcopy - L.ctab) / rpart, 64)) & ~1;
  }
  return o;
}


struct RunArgs {
  char* state;
  int n_steps;
  const int32_t* k;
  const double* new_pos;
  const uint8_t* accept;
  double* delta;
  double* djas;
  void* stream;
  RunPlan* plan;  // non-null: resolve the launch shape only, launch nothing
};

template <int DIM, bool MIXED, int NT, int SPT, int PPR, bool JAS, int PD, bool ORTHO, bool XTRA>
int run_inst(const LaunchBatch& b, const RunArgs& a) {
  auto* kern = k_run<DIM, MIXED, NT, SPT, PPR, JAS, PD, ORTHO, XTRA>;
  static const int per_cu = blocks_per_cu(kern, NT);
  const size_t budget = RUN_LDS_BUDGET / size_t(per_cu);
  RunLds L{};
  int ch = b.run_chunk > 0 ? std::min(b.run_chunk, RUN_CHUNK) : RUN_CHUNK;
  size_t lds = run_layout<DIM, MIXED, NT, SPT>(b, ch, L);
  if (b.run_chunk <= 0)
    while (lds > budget && ch > 8) lds = run_layout<DIM, MIXED, NT, SPT>(b, --ch, L);
  while (lds > RUN_LDS_BUDGET && ch > 1) lds = run_layout<DIM, MIXED, NT, SPT>(b, --ch, L);
  if (lds > RUN_LDS_BUDGET) return RUN_NO_FIT;
  if (a.plan) {
    *a.plan = RunPlan{1, NT, SPT, PPR, ch, ORTHO ? 0 : 1, int(lds), per_cu};
    return 0;
  }
  if (int rc = allow_lds(kern, lds)) return rc;
  hipLaunchKernelGGL(kern, dim3(b.n_walkers), dim3(NT), lds, as_stream(a.stream), b.d_sys, b.d_walk, a.state,
                     a.n_steps, b.n_walkers, a.k, a.new_pos, a.accept, a.delta, a.djas, L);
  return last_launch();
}

// Workgroup shapes of the fused kernel (threads NT, segments per thread SPT)
// by the largest segment count of the batch; `threads` picks among the
// shapes available for that count (0: the default, the first listed).
//   <= 256 segments: (256, 1)      <= 512: (256, 2)
//   <= 1024: (1024, 1) or (512, 2)  <= 2048: (512, 4)
// Particles per thread in registers: 1 when the largest walker has at most
// NT particles (always with 1024 threads, where larger walkers' remaining
// particles are read from LDS), else 2.
int run_shape(int max_n_seg, int max_particles, int threads, int* nt, int* spt, int* ppr) {
  struct Shape { int lim, nt, spt; };
  static const Shape shapes[] = {{256, 256, 1}, {512, 256, 2}, {1024, 1024, 1}, {1024, 512, 2}, {2048, 512, 4}};
  int lim = 0;
  for (const Shape& sh : shapes) {
    if (max_n_seg > sh.lim) continue;
    if (lim == 0) lim = sh.lim;
    if (sh.lim != lim) break;
    if (threads == 0 || threads == sh.nt) {
      *nt = sh.nt;
      *spt = sh.spt;
      *ppr = (sh.nt >= 1024 || max_particles <= sh.nt) ? 1 : 2;
      return 1;
    }
  }
  return 0;
}

template <int DIM, bool MIXED, bool JAS, int PD, bool ORTHO>
int run_jp(const LaunchBatch& b, const RunArgs& a) {
  static_assert(RUN_CHUNK <= 256, "staging uses one thread per move");
  int nt = 0, spt = 0, ppr = 0;
  if (!run_shape(b.max_n_seg, b.max_particles, b.run_threads, &nt, &spt, &ppr)) return RUN_NO_FIT;
  // XTRA: particles beyond the registers' share, or fixed ions, in some
  // walker.  Leaving those loops out pays at 512 and 1024 threads; the
  // 256-thread kernels keep them (without them the compiler spends more
  // registers there and runs slower).
  const bool xtra = b.max_particles > ppr * nt || b.max_fixed > 0;
#define EW_RUN(NT, SPT, PPR) \
  if (nt == NT && spt == SPT && ppr == PPR) return run_inst<DIM, MIXED, NT, SPT, PPR, JAS, PD, ORTHO, true>(b, a)
#define EW_RUN_X(NT, SPT, PPR)                                                                          \
  if (nt == NT && spt == SPT && ppr == PPR)                                                            \
    return xtra ? run_inst<DIM, MIXED, NT, SPT, PPR, JAS, PD, ORTHO, true>(b, a)                       \
                : run_inst<DIM, MIXED, NT, SPT, PPR, JAS, PD, ORTHO, false>(b, a)
  EW_RUN(256, 1, 1);
  EW_RUN(256, 1, 2);
  EW_RUN(256, 2, 1);
  EW_RUN(256, 2, 2);
  EW_RUN_X(1024, 1, 1);
  EW_RUN_X(512, 2, 2);
  EW_RUN_X(512, 4, 2);
#undef EW_RUN_X
#undef EW_RUN
  return RUN_NO_FIT;
}

template <int DIM, bool MIXED, bool JAS, int PD>
int run_jpo(const LaunchBatch& b, const RunArgs& a) {
  return b.all_ortho && !b.general_frame ? run_jp<DIM, MIXED, JAS, PD, true>(b, a)
                                         : run_jp<DIM, MIXED, JAS, PD, false>(b, a);
}

template <int DIM, bool MIXED>
int run_dim(const LaunchBatch& b, const RunArgs& a) {
  const bool jas = b.has_jastrow != 0, p16 = b.poly_deg <= 16;
  if (jas) return p16 ? run_jpo<DIM, MIXED, true, 16>(b, a) : run_jpo<DIM, MIXED, true, 32>(b, a);
  return p16 ? run_jpo<DIM, MIXED, false, 16>(b, a) : run_jpo<DIM, MIXED, false, 32>(b, a);
}

int run_any(const LaunchBatch& b, const RunArgs& a) {
  if (!b.all_wtab_lds) return RUN_NO_FIT;
  if (b.dim == 3) return b.mixed ? run_dim<3, true>(b, a) : run_dim<3, false>(b, a);
  return b.mixed ? run_dim<2, true>(b, a) : run_dim<2, false>(b, a);
}

}  // namespace

int launch_energy(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
                  void* stream) {
  return b.dim == 3 ? energy_dim<3>(b, pos, state, energy, jastrow, stream)
                   : energy_dim<2>(b, pos, state, energy, jastrow, stream);
}

int launch_delta(const LaunchBatch& b, char* state, const int32_t* k, const double* new_pos, double* delta,
                 double* djas, void* stream) {
  if (b.dim == 3) return b.mixed ? delta_dim<3, true>(b, state, k, new_pos, delta, djas, stream)
                                 : delta_dim<3, false>(b, state, k, new_pos, delta, djas, stream);
  return b.mixed ? delta_dim<2, true>(b, state, k, new_pos, delta, djas, stream)
                 : delta_dim<2, false>(b, state, k, new_pos, delta, djas, stream);
}

int launch_accept(const LaunchBatch& b, char* state, const uint8_t* accept, void* stream) {
  if (b.dim == 3) return b.mixed ? accept_dim<3, true>(b, state, accept, stream) : accept_dim<3, false>(b, state, accept, stream);
  return b.mixed ? accept_dim<2, true>(b, state, accept, stream) : accept_dim<2, false>(b, state, accept, stream);
}

int launch_run(const LaunchBatch& b, char* state, int n_steps, const int32_t* k, const double* new_pos,
               const uint8_t* accept, double* delta, double* djas, void* stream) {
  int rc = run_any(b, RunArgs{state, n_steps, k, new_pos, accept, delta, djas, stream, nullptr});
  if (rc != RUN_NO_FIT) return rc;
  // a shell table or walker too large for LDS: the same sequence through the per-step kernels
  const size_t W = size_t(b.n_walkers);
  for (int m = 0; m < n_steps; ++m) {
    rc = launch_delta(b, state, k + m * W, new_pos + m * W * b.dim, delta + m * W, djas ? djas + m * W : nullptr,
                      stream);
    if (!rc) rc = launch_accept(b, state, accept + m * W, stream);
    if (rc) return rc;
  }
  return 0;
}

void plan_run(const LaunchBatch& b, RunPlan* plan) {
  *plan = RunPlan{};
  if (run_any(b, RunArgs{nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, plan}) != 0) *plan = RunPlan{};
}

bool run_threads_valid(int max_n_seg, int threads) {
  int nt, spt, ppr;
  return threads == 0 || run_shape(max_n_seg, 0, threads, &nt, &spt, &ppr);
}

int time_run(const LaunchBatch& b, char* state, int n_steps, const int32_t* k, const double* new_pos,
             const uint8_t* accept, double* delta, void* stream, int reps, float* best_ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return int(hipErrorOutOfMemory);
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return int(hipErrorOutOfMemory);
  }
  int rc = launch_run(b, state, n_steps, k, new_pos, accept, delta, nullptr, stream);  // warm-up
  float best = 0.f;
  for (int r = 0; r < reps && !rc; ++r) {
    hipEventRecord(e0, as_stream(stream));
    rc = launch_run(b, state, n_steps, k, new_pos, accept, delta, nullptr, stream);
    hipEventRecord(e1, as_stream(stream));
    if (!rc) rc = int(hipEventSynchronize(e1));
    float ms = 0.f;
    if (!rc) rc = int(hipEventElapsedTime(&ms, e0, e1));
    if (!rc && (r == 0 || ms < best)) best = ms;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *best_ms = best;
  return rc;
}

int dev_arch(char* buf, int len) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return int(e);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return int(e);
  std::snprintf(buf, size_t(len), "%s", prop.gcnArchName);
  return 0;
}

int dev_copy(void* dst, const void* src, size_t bytes) {
  hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToDevice);
  return e == hipSuccess ? 0 : int(e);
}

int dev_memset(void* p, int value, size_t bytes) {
  hipError_t e = hipMemset(p, value, bytes);
  return e == hipSuccess ? 0 : int(e);
}

int dev_alloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  return e == hipSuccess ? 0 : int(e);
}
int dev_free(void* p) { return int(hipFree(p)); }
int dev_upload(void* dst, const void* src, size_t bytes) {
  hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  return e == hipSuccess ? 0 : int(e);
}
int dev_current(int* device) {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return int(e);
  if (count < 1) return int(hipErrorNoDevice);
  e = hipGetDevice(device);
  return e == hipSuccess ? 0 : int(e);
}
const char* dev_error_string(int code) { return hipGetErrorString(hipError_t(code)); }

}  // namespace ewald
