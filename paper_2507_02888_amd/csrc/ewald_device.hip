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

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "ewald_internal.h"

namespace ewald {

template <typename R>
struct cplx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
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

// exp(2 pi i n s) from the reduced phase frac(n s) in [-1/2, 1/2].
__device__ __forceinline__ cplx<double> phase(double s, int n, double) {
  double x = double(n) * s;
  x -= rint(x);
  double sn, cs;
  sincospi(2.0 * x, &sn, &cs);
  return {cs, sn};
}
__device__ __forceinline__ cplx<float> phase(double s, int n, float) {
  double x = double(n) * s;
  x -= rint(x);
  float sn, cs;
  sincospif(float(2.0 * x), &sn, &cs);
  return {cs, sn};
}

// Squared minimum-image distance between fractional positions a and b:
// reduce the fractional difference to [-1/2, 1/2], go Cartesian, then compare
// with the candidate images r0 +- v_c (|r0 +- v|^2 = |r0|^2 + |v|^2 -+ 2 r0.v).
template <int DIM>
__device__ __forceinline__ double min_r2(const double* a, const double* b, const DevSys* __restrict__ S,
                                         int n_cand) {
  double f[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    f[d] = a[d] - b[d];
    f[d] -= rint(f[d]);
  }
  double r[DIM];
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    double v = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) v = fma(f[d], S->A[d * 3 + e], v);
    r[e] = v;
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

// Pair potential accumulator phi(r) = erfc(alpha r)/r for r^2 < rc2.
// FP64 form: one FP64 sum.  Mixed form: phi = 1/r - erf(alpha r)/r with 1/r
// in FP64 (it carries the close-pair singularity) and the bounded erf part in
// FP32 with a Kahan sum.
template <bool MIXED>
struct PairAcc;

template <>
struct PairAcc<false> {
  double s = 0.0;
  __device__ __forceinline__ void add(double q, double r2, double alpha, double rc2) {
    if (r2 < rc2) {
      double r = sqrt(r2);
      s = fma(q, erfc(alpha * r) / r, s);
    }
  }
  __device__ __forceinline__ void sub(double q, double r2, double alpha, double rc2) { add(-q, r2, alpha, rc2); }
  __device__ __forceinline__ double value() const { return s; }
};

template <>
struct PairAcc<true> {
  double inv = 0.0;
  Kahan erfpart;
  __device__ __forceinline__ void add(double q, double r2, double alpha, double rc2) {
    if (r2 < rc2) {
      double ir = rsqrt(r2);
      inv = fma(q, ir, inv);
      float rf = float(r2 * ir);
      erfpart.add(float(q) * (erff(float(alpha) * rf) * float(ir)));
    }
  }
  __device__ __forceinline__ void sub(double q, double r2, double alpha, double rc2) { add(-q, r2, alpha, rc2); }
  __device__ __forceinline__ double value() const { return inv - erfpart.value(); }
};

// Sum NV values over the workgroup; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * (BLOCK / 64) + wv] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < BLOCK / 64; ++k) t += red[i * (BLOCK / 64) + k];
      v[i] = t;
    }
}

// Per-dimension phase tables of one position, n in [-nm, nm]:
// tab[d * (2 nm + 1) + nm + n] = exp(2 pi i n s_d).  Entries are written by
// threads [t0, t0 + DIM (nm + 1)) of the calling group.
template <int DIM, typename R>
__device__ __forceinline__ void fill_tables(cplx<R>* tab, const double* s, int nm, int e) {
  const int per = nm + 1;
  if (e >= 0 && e < DIM * per) {
    const int d = e / per, m = e - d * per;
    cplx<R> c = phase(s[d], m, R(0));
    const int tbl = 2 * nm + 1;
    tab[d * tbl + nm + m] = c;
    tab[d * tbl + nm - m] = {c.x, -c.y};
  }
}

// First phase of segment `pn` from the tables.
template <int DIM, typename R>
__device__ __forceinline__ cplx<R> anchor(const cplx<R>* tab, uint32_t pn, int nm) {
  const int tbl = 2 * nm + 1;
  cplx<R> e = cmul(tab[nm + unpack_n(pn, 0)], tab[tbl + nm + unpack_n(pn, 1)]);
  if (DIM == 3) e = cmul(e, tab[2 * tbl + nm + unpack_n(pn, 2)]);
  return e;
}

// Rebuild rho over the segments segs[i] = seg0 + i * BLOCK (i < NS) of one
// walker in FP64: rho = rho_fix + sum_p q_p exp(i G.r_p), particles taken
// TILE_P at a time through LDS phase tables (tabs: TILE_P * DIM * (2nm+1)).
// `pos` may point to global or LDS memory.  All threads must call it.
template <int DIM, int NS>
__device__ void rebuild_rho(cplx<double> (&acc)[NS][SEG], const uint32_t (&an)[NS], int seg0,
                            const DevSys* __restrict__ S, const double* pos, const double* q, int n,
                            cplx<double>* tabs) {
  const int nseg = S->n_seg, nm = S->nm, tbl = 2 * nm + 1;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int s = seg0 + i * BLOCK;
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
  for (int p0 = 0; p0 < n; p0 += TILE_P) {
    const int np = min(TILE_P, n - p0);
    for (int e = threadIdx.x; e < np * DIM * (nm + 1); e += BLOCK) {
      const int p = e / (DIM * (nm + 1));
      double sp[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) sp[d] = pos[(p0 + p) * DIM + d];
      fill_tables<DIM, double>(tabs + p * DIM * tbl, sp, nm, e - p * DIM * (nm + 1));
    }
    __syncthreads();
    for (int p = 0; p < np; ++p) {
      const cplx<double>* tp = tabs + p * DIM * tbl;
      const double qp = q[p0 + p];
      const cplx<double> u = tp[(DIM - 1) * tbl + nm + 1];
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        if (seg0 + i * BLOCK < nseg) {
          cplx<double> e = anchor<DIM, double>(tp, an[i], nm);
#pragma unroll
          for (int j = 0; j < SEG; ++j) {
            acc[i][j].x = fma(qp, e.x, acc[i][j].x);
            acc[i][j].y = fma(qp, e.y, acc[i][j].y);
            e = cmul(e, u);
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Energy: wrap positions, rho in FP64, reciprocal and Jastrow sums, real-space
// pairs, constants.  SPT = segments per thread held in registers.
template <int DIM, bool MIXED, int SPT>
__global__ __launch_bounds__(BLOCK) void k_energy(const DevSys* __restrict__ systems,
                                                  const DevWalker* __restrict__ walkers,
                                                  const double* __restrict__ pos, char* __restrict__ state,
                                                  double* __restrict__ energy, double* __restrict__ jastrow,
                                                  int lds_pos) {
  extern __shared__ double smem[];
  const int w = blockIdx.x, tid = threadIdx.x;
  const DevWalker W = walkers[w];
  const DevSys* __restrict__ S = systems + W.sys;
  const int n = W.n_mobile, nseg = S->n_seg, nfix = S->n_fixed, n_cand = S->n_cand;
  char* st = state + W.state_off;
  WalkerHdr* hdr = reinterpret_cast<WalkerHdr*>(st);
  double* spos = reinterpret_cast<double*>(st + HDR_BYTES);
  double* rho = reinterpret_cast<double*>(st + HDR_BYTES + walker_pos_bytes(n, DIM));
  double* lpos = smem;                       // [n][DIM]
  double* lq = smem + lds_pos * DIM;         // [n]
  double* red = lq + lds_pos;                // [4 * 4]
  cplx<double>* tabs = reinterpret_cast<cplx<double>*>(red + 16);

  const double* pw = pos + size_t(W.pos_off) * DIM;
  for (int i = tid; i < n; i += BLOCK) {
    double r[DIM], s[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) r[d] = pw[i * DIM + d];
    to_frac<DIM>(r, S->Ainv, s);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      lpos[i * DIM + d] = s[d];
      spos[i * DIM + d] = s[d];
    }
    lq[i] = S->mobile_q[i];
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
  rebuild_rho<DIM, SPT>(acc, an, tid, S, lpos, lq, n, tabs);
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
  // cyclically, plus i+n/2 for i < n/2 when n is even), then mobile-ion pairs
  const double alpha = S->alpha, rc2 = S->rc2;
  PairAcc<MIXED> pr;
  const int half = (n - 1) / 2;
  for (int i = tid; i < n; i += BLOCK) {
    double si[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) si[d] = lpos[i * DIM + d];
    const double qi = lq[i];
    for (int m = 1; m <= half; ++m) {
      int j = i + m;
      if (j >= n) j -= n;
      pr.add(qi * lq[j], min_r2<DIM>(si, lpos + j * DIM, S, n_cand), alpha, rc2);
    }
    if ((n & 1) == 0 && i < n / 2) {
      const int j = i + n / 2;
      pr.add(qi * lq[j], min_r2<DIM>(si, lpos + j * DIM, S, n_cand), alpha, rc2);
    }
    for (int I = 0; I < nfix; ++I)
      pr.add(qi * S->fixed_q[I], min_r2<DIM>(si, S->fixed_s + I * DIM, S, n_cand), alpha, rc2);
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
template <int DIM, bool MIXED>
__global__ __launch_bounds__(BLOCK) void k_delta(const DevSys* __restrict__ systems,
                                                 const DevWalker* __restrict__ walkers, char* __restrict__ state,
                                                 const int32_t* __restrict__ kk, const double* __restrict__ new_pos,
                                                 double* __restrict__ delta, double* __restrict__ djas) {
  using R = typename std::conditional<MIXED, float, double>::type;
  extern __shared__ double smem[];
  const int w = blockIdx.x, tid = threadIdx.x;
  const DevWalker W = walkers[w];
  const DevSys* __restrict__ S = systems + W.sys;
  const int n = W.n_mobile, nseg = S->n_seg, nm = S->nm, nfix = S->n_fixed, n_cand = S->n_cand;
  const int tbl = 2 * nm + 1;
  char* st = state + W.state_off;
  WalkerHdr* hdr = reinterpret_cast<WalkerHdr*>(st);
  const double* spos = reinterpret_cast<const double*>(st + HDR_BYTES);
  const double* rho = reinterpret_cast<const double*>(st + HDR_BYTES + walker_pos_bytes(n, DIM));
  double* red = smem;
  cplx<R>* to = reinterpret_cast<cplx<R>*>(smem + 16);
  cplx<R>* tn = to + DIM * tbl;

  const int k = kk[w];
  if (k < 0 || k >= n) {
    if (tid == 0) {
      delta[w] = NAN;
      if (djas) djas[w] = NAN;
      hdr->pending_k = -1;
    }
    return;
  }
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
  for (int e = tid; e < 2 * DIM * (nm + 1); e += BLOCK) {
    if (e < DIM * (nm + 1)) fill_tables<DIM, R>(to, so, nm, e);
    else fill_tables<DIM, R>(tn, sn, nm, e - DIM * (nm + 1));
  }
  __syncthreads();

  // reciprocal space: t(G) = 2 q Re(conj(rho) d) + q^2 |d|^2, d = e_new - e_old
  const cplx<R> uo = to[(DIM - 1) * tbl + nm + 1], un = tn[(DIM - 1) * tbl + nm + 1];
  const double* __restrict__ wt = S->w;
  const double* __restrict__ ja = S->ja;
  double accE64 = 0.0, accJ64 = 0.0;
  Kahan accE32, accJ32;
  const R q = R(qk), q2 = R(qk * qk);
  for (int s = tid; s < nseg; s += BLOCK) {
    const uint32_t pn = S->seg_n[s];
    cplx<R> eo = anchor<DIM, R>(to, pn, nm);
    cplx<R> en = anchor<DIM, R>(tn, pn, nm);
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const size_t g = size_t(j) * nseg + s;
      const R dx = en.x - eo.x, dy = en.y - eo.y;
      const R rx = R(rho[2 * g]), ry = R(rho[2 * g + 1]);
      const R t = R(2) * q * (rx * dx + ry * dy) + q2 * (dx * dx + dy * dy);
      if (MIXED) {
        accE32.add(float(wt[g]) * float(t));
        if (ja) accJ32.add(float(ja[g]) * float(t));
      } else {
        accE64 = fma(wt[g], double(t), accE64);
        if (ja) accJ64 = fma(ja[g], double(t), accJ64);
      }
      eo = cmul(eo, uo);
      en = cmul(en, un);
    }
  }
  // real space
  const double alpha = S->alpha, rc2 = S->rc2;
  PairAcc<MIXED> pr;
  for (int j = tid; j < n; j += BLOCK) {
    if (j == k) continue;
    const double* sj = spos + j * DIM;
    const double qj = S->mobile_q[j];
    pr.add(qj, min_r2<DIM>(sn, sj, S, n_cand), alpha, rc2);
    pr.sub(qj, min_r2<DIM>(so, sj, S, n_cand), alpha, rc2);
  }
  for (int I = tid; I < nfix; I += BLOCK) {
    const double* sj = S->fixed_s + I * DIM;
    const double qj = S->fixed_q[I];
    pr.add(qj, min_r2<DIM>(sn, sj, S, n_cand), alpha, rc2);
    pr.sub(qj, min_r2<DIM>(so, sj, S, n_cand), alpha, rc2);
  }
  double v[2] = {(MIXED ? accE32.value() : accE64) + qk * pr.value(), MIXED ? accJ32.value() : accJ64};
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
  const int w = blockIdx.x, tid = threadIdx.x;
  const DevWalker W = walkers[w];
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
    for (int e = tid; e < 2 * DIM * (nm + 1); e += BLOCK) {
      if (e < DIM * (nm + 1)) fill_tables<DIM, R>(to, so, nm, e);
      else fill_tables<DIM, R>(tn, sn, nm, e - DIM * (nm + 1));
    }
  }
  __syncthreads();  // every thread has read the header and pending position
  if (acc) {
    const R q = R(S->mobile_q[pk]);
    const cplx<R> uo = to[(DIM - 1) * tbl + nm + 1], un = tn[(DIM - 1) * tbl + nm + 1];
    for (int s = tid; s < nseg; s += BLOCK) {
      const uint32_t pn = S->seg_n[s];
      cplx<R> eo = anchor<DIM, R>(to, pn, nm);
      cplx<R> en = anchor<DIM, R>(tn, pn, nm);
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const size_t g = size_t(j) * nseg + s;
        rho[2 * g] += double(q * (en.x - eo.x));
        rho[2 * g + 1] += double(q * (en.y - eo.y));
        eo = cmul(eo, uo);
        en = cmul(en, un);
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
  const int w = blockIdx.x, chunk = blockIdx.y, tid = threadIdx.x;
  const DevWalker W = walkers[w];
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
// Fused multi-move: n_steps proposals per walker with rho, weights and the
// segment anchors in registers and positions in LDS for the whole sequence.
template <int DIM, bool MIXED, int SPT, bool JAS>
__global__ __launch_bounds__(BLOCK) void k_run(const DevSys* __restrict__ systems,
                                               const DevWalker* __restrict__ walkers, char* __restrict__ state,
                                               int n_steps, int n_walkers, const int32_t* __restrict__ kk,
                                               const double* __restrict__ new_pos, const uint8_t* __restrict__ accept,
                                               double* __restrict__ delta, double* __restrict__ djas, int lds_pos,
                                               int lds_tab) {
  using R = typename std::conditional<MIXED, float, double>::type;
  extern __shared__ double smem[];
  const int w = blockIdx.x, tid = threadIdx.x;
  const DevWalker W = walkers[w];
  const DevSys* __restrict__ S = systems + W.sys;
  const int n = W.n_mobile, nseg = S->n_seg, nm = S->nm, nfix = S->n_fixed, n_cand = S->n_cand;
  const int K = S->refresh_every, tbl = 2 * nm + 1;
  // the mixed form multiplies weights with FP32 terms, so it keeps them in FP32
  using WT = R;
  char* st = state + W.state_off;
  WalkerHdr* hdr = reinterpret_cast<WalkerHdr*>(st);
  double* spos = reinterpret_cast<double*>(st + HDR_BYTES);
  double* rho = reinterpret_cast<double*>(st + HDR_BYTES + walker_pos_bytes(n, DIM));
  double* lpos = smem;                  // [n][DIM]
  double* lq = smem + lds_pos * DIM;    // [n]
  double* red = lq + lds_pos;           // 16
  cplx<R>* to = reinterpret_cast<cplx<R>*>(red + 16);
  cplx<R>* tn = to + DIM * tbl;
  cplx<double>* tabs = reinterpret_cast<cplx<double>*>(red + 16 + lds_tab);  // rebuild tiles

  for (int i = tid; i < n * DIM; i += BLOCK) lpos[i] = spos[i];
  for (int i = tid; i < n; i += BLOCK) lq[i] = S->mobile_q[i];
  int counter = hdr->counter;
  int n_acc = hdr->n_accepts, n_ref = hdr->n_refresh;
  double drift = hdr->drift_max;
  if (K > 0 && counter >= K) counter = 0;

  uint32_t an[SPT];
  cplx<double> rv[SPT][SEG];
  WT wv[SPT][SEG], av[SPT][SEG];
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    const int s = tid + i * BLOCK;
    an[i] = s < nseg ? S->seg_n[s] : 0u;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const size_t g = size_t(j) * nseg + s;
      rv[i][j] = s < nseg ? cplx<double>{rho[2 * g], rho[2 * g + 1]} : cplx<double>{0.0, 0.0};
      wv[i][j] = s < nseg ? WT(S->w[g]) : WT(0);
      av[i][j] = (JAS && s < nseg) ? WT(S->ja[g]) : WT(0);
    }
  }
  __syncthreads();

  const double alpha = S->alpha, rc2 = S->rc2;
  for (int m = 0; m < n_steps; ++m) {
    const size_t idx = size_t(m) * n_walkers + w;
    const int k = kk[idx];
    if (k < 0 || k >= n) {  // uniform
      if (tid == 0) {
        delta[idx] = NAN;
        if (djas) djas[idx] = NAN;
      }
      continue;
    }
    const bool acc = accept[idx] != 0;
    double sn[DIM], so[DIM];
    {
      double r[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) r[d] = new_pos[idx * DIM + d];
      to_frac<DIM>(r, S->Ainv, sn);
#pragma unroll
      for (int d = 0; d < DIM; ++d) so[d] = lpos[k * DIM + d];
    }
    const double qk = lq[k];
    for (int e = tid; e < 2 * DIM * (nm + 1); e += BLOCK) {
      if (e < DIM * (nm + 1)) fill_tables<DIM, R>(to, so, nm, e);
      else fill_tables<DIM, R>(tn, sn, nm, e - DIM * (nm + 1));
    }
    __syncthreads();

    const cplx<R> uo = to[(DIM - 1) * tbl + nm + 1], un = tn[(DIM - 1) * tbl + nm + 1];
    const R q = R(qk), q2 = R(qk * qk);
    double accE64 = 0.0, accJ64 = 0.0;
    Kahan accE32, accJ32;
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      if (tid + i * BLOCK < nseg) {
        cplx<R> eo = anchor<DIM, R>(to, an[i], nm);
        cplx<R> en = anchor<DIM, R>(tn, an[i], nm);
#pragma unroll
        for (int j = 0; j < SEG; ++j) {
          const R dx = en.x - eo.x, dy = en.y - eo.y;
          const R t = R(2) * q * (R(rv[i][j].x) * dx + R(rv[i][j].y) * dy) + q2 * (dx * dx + dy * dy);
          if (MIXED) {
            accE32.add(float(wv[i][j]) * float(t));
            if (JAS) accJ32.add(float(av[i][j]) * float(t));
          } else {
            accE64 = fma(wv[i][j], double(t), accE64);
            if (JAS) accJ64 = fma(av[i][j], double(t), accJ64);
          }
          if (acc) {
            rv[i][j].x += double(q * dx);
            rv[i][j].y += double(q * dy);
          }
          eo = cmul(eo, uo);
          en = cmul(en, un);
        }
      }
    }
    PairAcc<MIXED> pr;
    for (int j = tid; j < n; j += BLOCK) {
      if (j == k) continue;
      const double* sj = lpos + j * DIM;
      const double qj = lq[j];
      pr.add(qj, min_r2<DIM>(sn, sj, S, n_cand), alpha, rc2);
      pr.sub(qj, min_r2<DIM>(so, sj, S, n_cand), alpha, rc2);
    }
    for (int I = tid; I < nfix; I += BLOCK) {
      const double* sj = S->fixed_s + I * DIM;
      const double qj = S->fixed_q[I];
      pr.add(qj, min_r2<DIM>(sn, sj, S, n_cand), alpha, rc2);
      pr.sub(qj, min_r2<DIM>(so, sj, S, n_cand), alpha, rc2);
    }
    double v[2] = {(MIXED ? accE32.value() : accE64) + qk * pr.value(), MIXED ? accJ32.value() : accJ64};
    block_sum<2>(v, red);
    if (tid == 0) {
      delta[idx] = v[0];
      if (djas) djas[idx] = v[1];
      if (acc)
#pragma unroll
        for (int d = 0; d < DIM; ++d) lpos[k * DIM + d] = sn[d];
    }
    if (acc) {
      counter += 1;
      n_acc += 1;
    }
    __syncthreads();
    if (MIXED && K > 0 && counter >= K) {  // uniform
      // park the running rho in the state, rebuild in registers, compare
#pragma unroll
      for (int i = 0; i < SPT; ++i) {
        const int s = tid + i * BLOCK;
        if (s < nseg)
#pragma unroll
          for (int j = 0; j < SEG; ++j) {
            const size_t g = size_t(j) * nseg + s;
            rho[2 * g] = rv[i][j].x;
            rho[2 * g + 1] = rv[i][j].y;
          }
      }
      rebuild_rho<DIM, SPT>(rv, an, tid, S, lpos, lq, n, tabs);
      double dm = 0.0;
#pragma unroll
      for (int i = 0; i < SPT; ++i) {
        const int s = tid + i * BLOCK;
        if (s < nseg)
#pragma unroll
          for (int j = 0; j < SEG; ++j) {
            const size_t g = size_t(j) * nseg + s;
            dm = fmax(dm, fmax(fabs(rv[i][j].x - rho[2 * g]), fabs(rv[i][j].y - rho[2 * g + 1])));
          }
      }
      for (int off = 32; off > 0; off >>= 1) dm = fmax(dm, __shfl_xor(dm, off, 64));
      if ((tid & 63) == 0) red[8 + (tid >> 6)] = dm;
      __syncthreads();
      for (int k2 = 0; k2 < BLOCK / 64; ++k2) drift = fmax(drift, red[8 + k2]);
      __syncthreads();
      counter = 0;
      n_ref += 1;
    }
  }

  // write back
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    const int s = tid + i * BLOCK;
    if (s < nseg)
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const size_t g = size_t(j) * nseg + s;
        rho[2 * g] = rv[i][j].x;
        rho[2 * g + 1] = rv[i][j].y;
      }
  }
  for (int i = tid; i < n * DIM; i += BLOCK) spos[i] = lpos[i];
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

template <int DIM, bool MIXED>
int energy_dim(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
               void* stream) {
  const int lds_pos = even(b.max_particles);
  const size_t tab = size_t(TILE_P) * DIM * (2 * b.max_nm + 1) * sizeof(cplx<double>);
  const size_t lds = size_t(lds_pos) * (DIM + 1) * 8 + 16 * 8 + tab;
  dim3 grid(b.n_walkers), block(BLOCK);
  hipStream_t st = as_stream(stream);
  int rc = 0;
  switch (spt_for(b.max_n_seg)) {
    case 1: if (!(rc = allow_lds(k_energy<DIM, MIXED, 1>, lds))) hipLaunchKernelGGL((k_energy<DIM, MIXED, 1>), grid, block, lds, st, b.d_sys, b.d_walk, pos, state, energy, jastrow, lds_pos); break;
    case 2: if (!(rc = allow_lds(k_energy<DIM, MIXED, 2>, lds))) hipLaunchKernelGGL((k_energy<DIM, MIXED, 2>), grid, block, lds, st, b.d_sys, b.d_walk, pos, state, energy, jastrow, lds_pos); break;
    case 4: if (!(rc = allow_lds(k_energy<DIM, MIXED, 4>, lds))) hipLaunchKernelGGL((k_energy<DIM, MIXED, 4>), grid, block, lds, st, b.d_sys, b.d_walk, pos, state, energy, jastrow, lds_pos); break;
    default: if (!(rc = allow_lds(k_energy<DIM, MIXED, 8>, lds))) hipLaunchKernelGGL((k_energy<DIM, MIXED, 8>), grid, block, lds, st, b.d_sys, b.d_walk, pos, state, energy, jastrow, lds_pos); break;
  }
  return rc ? rc : last_launch();
}

template <int DIM, bool MIXED>
int delta_dim(const LaunchBatch& b, char* state, const int32_t* k, const double* new_pos, double* delta,
              double* djas, void* stream) {
  using R = typename std::conditional<MIXED, float, double>::type;
  const size_t lds = 16 * 8 + size_t(2) * DIM * (2 * b.max_nm + 1) * sizeof(cplx<R>);
  hipLaunchKernelGGL((k_delta<DIM, MIXED>), dim3(b.n_walkers), dim3(BLOCK), lds, as_stream(stream), b.d_sys,
                     b.d_walk, state, k, new_pos, delta, djas);
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

template <int DIM, bool MIXED, int SPT, bool JAS>
int run_inst(const LaunchBatch& b, char* state, int n_steps, const int32_t* k, const double* new_pos,
             const uint8_t* accept, double* delta, double* djas, void* stream) {
  using R = typename std::conditional<MIXED, float, double>::type;
  const int lds_pos = even(b.max_particles);
  const size_t mtab = size_t(2) * DIM * (2 * b.max_nm + 1) * sizeof(cplx<R>);
  const int lds_tab = even(int((mtab + 7) / 8));  // in doubles
  const size_t rtab = MIXED ? size_t(TILE_P) * DIM * (2 * b.max_nm + 1) * sizeof(cplx<double>) : 0;
  const size_t lds = size_t(lds_pos) * (DIM + 1) * 8 + 16 * 8 + size_t(lds_tab) * 8 + rtab;
  if (int rc = allow_lds(k_run<DIM, MIXED, SPT, JAS>, lds)) return rc;
  hipLaunchKernelGGL((k_run<DIM, MIXED, SPT, JAS>), dim3(b.n_walkers), dim3(BLOCK), lds, as_stream(stream),
                     b.d_sys, b.d_walk, state, n_steps, b.n_walkers, k, new_pos, accept, delta, djas, lds_pos,
                     lds_tab);
  return last_launch();
}

template <int DIM, bool MIXED>
int run_dim(const LaunchBatch& b, char* state, int n_steps, const int32_t* k, const double* new_pos,
            const uint8_t* accept, double* delta, double* djas, void* stream) {
  const bool jas = b.has_jastrow != 0;
  switch (spt_for(b.max_n_seg)) {
    case 1: return jas ? run_inst<DIM, MIXED, 1, true>(b, state, n_steps, k, new_pos, accept, delta, djas, stream)
                       : run_inst<DIM, MIXED, 1, false>(b, state, n_steps, k, new_pos, accept, delta, djas, stream);
    case 2: return jas ? run_inst<DIM, MIXED, 2, true>(b, state, n_steps, k, new_pos, accept, delta, djas, stream)
                       : run_inst<DIM, MIXED, 2, false>(b, state, n_steps, k, new_pos, accept, delta, djas, stream);
    case 4: return jas ? run_inst<DIM, MIXED, 4, true>(b, state, n_steps, k, new_pos, accept, delta, djas, stream)
                       : run_inst<DIM, MIXED, 4, false>(b, state, n_steps, k, new_pos, accept, delta, djas, stream);
    default: return jas ? run_inst<DIM, MIXED, 8, true>(b, state, n_steps, k, new_pos, accept, delta, djas, stream)
                        : run_inst<DIM, MIXED, 8, false>(b, state, n_steps, k, new_pos, accept, delta, djas, stream);
  }
}

}  // namespace

int launch_energy(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
                  void* stream) {
  if (b.dim == 3) return b.mixed ? energy_dim<3, true>(b, pos, state, energy, jastrow, stream)
                                 : energy_dim<3, false>(b, pos, state, energy, jastrow, stream);
  return b.mixed ? energy_dim<2, true>(b, pos, state, energy, jastrow, stream)
                 : energy_dim<2, false>(b, pos, state, energy, jastrow, stream);
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
  if (b.dim == 3) return b.mixed ? run_dim<3, true>(b, state, n_steps, k, new_pos, accept, delta, djas, stream)
                                 : run_dim<3, false>(b, state, n_steps, k, new_pos, accept, delta, djas, stream);
  return b.mixed ? run_dim<2, true>(b, state, n_steps, k, new_pos, accept, delta, djas, stream)
                 : run_dim<2, false>(b, state, n_steps, k, new_pos, accept, delta, djas, stream);
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
