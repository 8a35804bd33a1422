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
//
// This translation unit holds the energy, per-step delta/accept and rebuild
// kernels, the fused kernel's dispatch, and the device memory helpers; the
// fused kernels themselves are compiled in ewald_run_d*.hip.

#include <new>

#include "ewald_run.h"

namespace ewald {

// ---------------------------------------------------------------------------
// Energy: wrap positions, rho in FP64, reciprocal and Jastrow sums, real-space
// pairs, constants.  SPT = segments per thread held in registers.  Both
// precision forms compute the energy alike, in FP64: it adds ~N^2/4 pair terms
// of one sign (like charges), so any FP32 rounding bias of the pair function
// would add up coherently, while in a move delta it cancels between the old
// and new terms.  The pair loop works in the orthogonal-sublattice frame when
// the cell has one (ORTHO); rho is built from the fractional positions just
// stored in the walker state.
// UJ: the Jastrow value also takes the two-body polynomial term u over the
// mobile pairs (Sec. 2.3, Eq. (8)).
template <int DIM, int SPT, int PD, bool ORTHO, bool UJ>
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
  double* lpos = smem + 16;                  // [DIM][lds_pos] in the pair loop's geometry (planar:
                                             // lanes reading consecutive particles hit consecutive banks)
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
  // a layered 2D system (two planes): rho of each plane, with the
  // cross-plane term 2 w_x Re(rho_0 conj(rho_1)); the second plane's rho
  // follows the first in the state
  const bool lay = DIM == 2 && S->n_layers > 1;
  const int n0 = lay ? S->n0 : n;
  cplx<double> acc[SPT][SEG];
  rebuild_rho<DIM, SPT>(acc, an, tid, S, spos, S->mobile_q, n0, tabs, tile);
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
  if (lay) {
    cplx<double> acc1[SPT][SEG];
    rebuild_rho<DIM, SPT>(acc1, an, tid, S, spos + size_t(n0) * DIM, S->mobile_q + n0, n - n0, tabs, tile,
                          S->rho_fix1);
    double* rho1 = rho + 2 * size_t(SEG) * nseg;
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      const int s = tid + i * BLOCK;
      if (s < nseg) {
#pragma unroll
        for (int j = 0; j < SEG; ++j) {
          const size_t g = size_t(j) * nseg + s;
          const double m2 = acc1[i][j].x * acc1[i][j].x + acc1[i][j].y * acc1[i][j].y;
          const double x = acc[i][j].x * acc1[i][j].x + acc[i][j].y * acc1[i][j].y;
          er = fma(S->w[g], m2, er);
          er = fma(2.0 * S->wx[g], x, er);
          rho1[2 * g] = acc1[i][j].x;
          rho1[2 * g + 1] = acc1[i][j].y;
        }
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
    for (int d = 0; d < DIM; ++d) lpos[d * lds_pos + i] = x[d];
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
  double eu = 0.0;  // UJ: this thread's share of sum_{i<j} u(r_ij)
  for (int i = tid; i < n; i += BLOCK) {
    double si[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) si[d] = lpos[d * lds_pos + i];
    const double qi = lq[i];
    const int spi = UJ ? S->spin[i] : 0;
    const int li = i >= n0 ? 1 : 0;  // plane of particle i (layered systems)
    // the partners i + 1 .. i + half (cyclically), which every particle has:
    // the group bounds are the same for every lane and no partner is an ion
    for (int m0 = 0; m0 < half; m0 += 4) {
      double qq[4], r2[4], ir[4];
      bool uneq[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        int j = i + m0 + c + 1;
        if (j >= n) j -= n;
        if (m0 + c < half) {
          double sj[DIM];
#pragma unroll
          for (int d = 0; d < DIM; ++d) sj[d] = lpos[d * lds_pos + j];
          qq[c] = qi * lq[j];
          r2[c] = image_r2<DIM, ORTHO>(si, sj, S, n_cand, K);
          if (lay) r2[c] += ((j >= n0 ? 1 : 0) != li) ? S->dz2 : 0.0;
          uneq[c] = UJ && S->spin[j] != spi;
        } else {
          qq[c] = 0.0;
          r2[c] = rc2;
          uneq[c] = false;
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) ir[c] = rsqrt_pos(r2[c]);
      pr.template add_ir<4>(qq, r2, ir);
      if (UJ)
#pragma unroll
        for (int c = 0; c < 4; ++c) eu += u_pair(S, m0 + c < half, uneq[c], r2[c], ir[c]);
    }
    // then i + n/2 for i < n/2 when n is even, and every fixed ion
    const int n_mob = ((n & 1) == 0 && i < n / 2) ? 1 : 0;
    const int n_part = n_mob + nfix;
    for (int m0 = 0; m0 < n_part; m0 += 4) {
      double qq[4], r2[4], ir[4];
      bool mobc[4], uneq[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int m = m0 + c;
        const bool mob = m < n_mob, fix = !mob && m < n_part;
        int j = i + half + m + 1;
        if (j >= n) j -= n;
        double sj[DIM];
        if (mob) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) sj[d] = lpos[d * lds_pos + j];
        } else {
          geo_pos<DIM, ORTHO>(S->fixed_s + (fix ? m - n_mob : 0) * DIM, S, sj);
        }
        qq[c] = mob ? qi * lq[j] : fix ? qi * S->fixed_q[m - n_mob] : 0.0;
        r2[c] = (mob || fix) ? image_r2<DIM, ORTHO>(si, sj, S, n_cand, K) : rc2;
        if (lay && (mob || fix)) {
          const int lj = mob ? (j >= n0 ? 1 : 0) : S->fixed_layer[m - n_mob];
          r2[c] += lj != li ? S->dz2 : 0.0;
        }
        mobc[c] = mob;
        uneq[c] = UJ && mob && S->spin[j] != spi;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) ir[c] = rsqrt_pos(r2[c]);
      pr.template add_ir<4>(qq, r2, ir);
      if (UJ)
#pragma unroll
        for (int c = 0; c < 4; ++c) eu += u_pair(S, mobc[c], uneq[c], r2[c], ir[c]);
    }
  }
  double v[3] = {pr.value(), er, ej + eu};
  block_sum<3>(v, red);
  if (tid == 0) {
    energy[w] = v[0] + v[1] + S->e_const;
    if (jastrow) jastrow[w] = v[2];
  }
}

// ---------------------------------------------------------------------------
// Per-step calls: move delta (optionally folding in the previous move's
// accept) and accept.
constexpr int RED_DELTA = 48;  // LDS doubles for k_delta's reduction: up to 12 sums x 4 waves

// rho += q (e_new - e_old) for an accepted move: the difference and its
// product with q in the form's precision, the sum in FP64 (the per-step
// accept and the accept folded into the step kernel use this arithmetic,
// the fused sweep the same expression).
template <typename R>
__device__ __forceinline__ void add_move(double2& r, R q, const cplx<R>& en, const cplx<R>& eo) {
  r.x += double(q * (en.x - eo.x));
  r.y += double(q * (en.y - eo.y));
}

// Apply an accepted move to one plane's rho, streaming its segments once
// (to, tn: the old and new position's phase tables, already in LDS).
template <int DIM, typename R>
__device__ __forceinline__ void accept_stream(const DevSys* __restrict__ S, const cplx<R>* to, const cplx<R>* tn,
                                              double* rho, R q) {
  const int nseg = S->n_seg, nm = S->nm, tbl = 2 * nm + 1;
  const cplx<R> uo = tab_at(to, DIM - 1, nm + 1, tbl), un = tab_at(tn, DIM - 1, nm + 1, tbl);
  double2* rho2 = reinterpret_cast<double2*>(rho);
  for (int s = threadIdx.x; s < nseg; s += BLOCK) {
    double2 r[SEG];
#pragma unroll
    for (int j = 0; j < SEG; ++j) r[j] = rho2[size_t(j) * nseg + s];
    const uint32_t pn = S->seg_n[s];
    SegWalk<R> wo(anchor<DIM, R>(to, pn, nm), uo), wn(anchor<DIM, R>(tn, pn, nm), un);
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      add_move(r[j], q, wn.cur, wo.cur);
      rho2[size_t(j) * nseg + s] = r[j];
      if (j + 1 < SEG) {
        wo.step(j);
        wn.step(j);
      }
    }
  }
}

// Header side of an accept/reject (one thread): the position, the refresh
// counter (reset first when the previous call left it at K, i.e. rho was
// rebuilt after it) and the accept count; no move is pending afterwards.
template <int DIM>
__device__ __forceinline__ void accept_header(WalkerHdr* hdr, double* spos, int pk, bool acc, const double* sp,
                                              int K) {
  int counter = hdr->counter;
  if (K > 0 && counter >= K) counter = 0;
  if (acc) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) spos[pk * DIM + d] = sp[d];
    counter += 1;
    hdr->n_accepts += 1;
  }
  hdr->counter = counter;
  hdr->pending_k = -1;
}

// Move delta: dE and dJ of moving particle k to new_pos; records the pending
// move.  rho is streamed from the state once (slot-planar, coalesced).
//
// DER: also the gradient and Laplacian of J with respect to the moved
// particle at the proposed configuration (Sec. 2.3, Eq. (9); Sec. 5.2 offloads
// the values and derivatives of the p term).  With rho' = rho + q (e' - e_old)
// the proposed structure factor and z = conj(rho') e',
//   grad_k J = -2 q sum_H a G Im z,   lap_k J = -2 q sum_H a |G|^2 (Re z - q).
// G = sum_d n_d b_d, so the gradient is accumulated in reduced coordinates,
// S_d = sum_H a n_d Im z (per segment: the last index runs n_last + j), and
// turned into Cartesian components once per move; |G|^2 is constant on a
// shell and comes with a from the shell table.
// UJ: dJ also takes the two-body polynomial term u of the mobile pairs (and,
// with DER, its gradient and Laplacian at the new position).
//
// Step form (accept_prev != NULL): first the accept or reject of the move
// left pending by the previous call, with the arithmetic and header updates
// of k_accept, folded into this call's rho stream: rho is read once and, for
// an accepted move, written back updated, and the accepted particle's
// position is taken from the pending record; then the new move's delta from
// the updated rho and positions.  This saves the accept's second pass over
// rho.  In the FP32-mixed form a walker whose accept brings the refresh
// counter to K gets rho rebuilt by k_rebuild after this launch and its delta
// recomputed by a second launch with redo = 1, which leaves every other
// walker alone; the outputs are then those of k_accept + k_rebuild + k_delta.
template <int DIM, bool MIXED, int PD, bool DER, bool UJ>
__global__ __launch_bounds__(BLOCK, 4) void k_delta(const DevSys* __restrict__ systems,
                                                 const DevWalker* __restrict__ walkers, char* __restrict__ state,
                                                 const int32_t* __restrict__ kk, const double* __restrict__ new_pos,
                                                 double* __restrict__ delta, double* __restrict__ djas,
                                                 double* __restrict__ jgrad, double* __restrict__ jlap, int lds_tab,
                                                 const uint8_t* __restrict__ accept_prev, int redo) {
  using R = typename std::conditional<MIXED, float, double>::type;
  using WT2 = cplx<R>;  // (weight, Jastrow coefficient) in the form's precision
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
  if (redo && !(K > 0 && hdr->counter >= K)) return;  // uniform: redo only where rho was just rebuilt
  // the pending move's accept (step form)
  const int pk = hdr->pending_k;
  const bool acc = accept_prev != nullptr && pk >= 0 && pk < n && accept_prev[w] != 0;
  double sp[DIM];  // the accepted particle's new position
#pragma unroll
  for (int d = 0; d < DIM; ++d) sp[d] = acc ? hdr->pending_s[d] : 0.0;
  const R qp = acc ? R(S->mobile_q[pk]) : R(0);
  // layered 2D system: rho of plane 1 follows plane 0's
  const bool lay = DIM == 2 && S->n_layers > 1;
  const size_t plane = 2 * size_t(SEG) * nseg;
  const int lp = lay && acc && pk >= S->n0 ? 1 : 0;
  double* red = smem;  // [NV][4], NV <= RED_DELTA / 4
  cplx<R>* to = reinterpret_cast<cplx<R>*>(smem + RED_DELTA);
  cplx<R>* tn = to + DIM * tbl;
  cplx<R>* tpo = tn + DIM * tbl;  // the accepted move's old and new position
  cplx<R>* tpn = tpo + DIM * tbl;
  WT2* ltab = reinterpret_cast<WT2*>(smem + RED_DELTA + lds_tab);  // shell table (when it fits)
  R* ltab2 = reinterpret_cast<R*>(ltab + S->n_wtab);      // a |G|^2 per shell (DER)

  const int k = kk[w];
  if (k < 0 || k >= n) {
    if (acc) {  // the accept still applies
      double so_p[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) so_p[d] = spos[pk * DIM + d];
      if (tid < 2 * DIM) fill_row<R>(tpo + tid * tbl, pick_coord<DIM>(so_p, sp, tid), nm);
      __syncthreads();
      accept_stream<DIM, R>(S, tpo, tpn, rho + lp * plane, qp);
    }
    if (tid == 0) {
      delta[w] = NAN;
      if (djas) djas[w] = NAN;
      if (DER) {
        for (int d = 0; d < DIM; ++d) jgrad[size_t(w) * DIM + d] = NAN;
        jlap[w] = NAN;
      }
      if (accept_prev) accept_header<DIM>(hdr, spos, pk, acc, sp, K);
      hdr->pending_k = -1;
    }
    return;
  }
  const int lk = lay && k >= S->n0 ? 1 : 0;
  double2* __restrict__ rho2 = reinterpret_cast<double2*>(rho + lk * plane);
  double2* __restrict__ rhoo2 = reinterpret_cast<double2*>(rho + (1 - lk) * plane);  // the other plane (lay)
  const bool acc_own = acc && lp == lk;  // else the other plane's
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
    for (int i = tid; i < S->n_wtab; i += BLOCK) {
      ltab[i] = {R(S->wa_tab[2 * i]), R(S->wa_tab[2 * i + 1])};
      if (DER) ltab2[i] = R(S->jg2_tab[i]);
    }
  double sn[DIM], so[DIM];
  {
    double r[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) r[d] = new_pos[size_t(w) * DIM + d];
    to_frac<DIM>(r, S->Ainv, sn);
    const bool same = acc && k == pk;  // moving the particle just accepted: from its new position
    // the move's positions are the same in every lane: scalar registers
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      sn[d] = uniform_d(sn[d]);
      so[d] = uniform_d(same ? sp[d] : spos[k * DIM + d]);
      sp[d] = uniform_d(sp[d]);
    }
  }
  const double qk = S->mobile_q[k];
  if (tid < 2 * DIM) fill_row<R>(to + tid * tbl, pick_coord<DIM>(so, sn, tid), nm);  // to, then tn
  if (acc && tid >= 2 * DIM && tid < 4 * DIM) {
    double so_p[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) so_p[d] = spos[pk * DIM + d];
    fill_row<R>(tpo + (tid - 2 * DIM) * tbl, pick_coord<DIM>(so_p, sp, tid - 2 * DIM), nm);  // tpo, then tpn
  }
  __syncthreads();

  // reciprocal space: t(G) = 2 q Re(conj(rho) d) + q^2 |d|^2, d = e_new - e_old
  // the walks' steps exp(2 pi i s_last) are the same in every lane: kept in scalar registers
  auto ustep = [&](const cplx<R>* t) {
    const cplx<R> u = tab_at(t, DIM - 1, nm + 1, tbl);
    return cplx<R>{uniform_r(u.x), uniform_r(u.y)};
  };
  const cplx<R> uo = ustep(to), un = ustep(tn), upo = ustep(tpo), upn = ustep(tpn);
  const R c2o = uniform_r(R(2) * uo.x), c2n = uniform_r(R(2) * un.x);
  const R c2po = uniform_r(R(2) * upo.x), c2pn = uniform_r(R(2) * upn.x);
  const double* __restrict__ wt = S->w;
  const double* __restrict__ ja = S->ja;
  // t(G) = q^2 [dx (dx + (2/q) rho_x) + dy (dy + (2/q) rho_y)]: q^2 is applied
  // once to the sums, and a neutral particle's move changes nothing
  double accE64 = 0.0, accJ64 = 0.0, accX64 = 0.0;
  Kahan accE32, accJ32, accX32;  // X: the cross-plane sum of a layered system, sum_H w_x Re(conj(rho_o) d)
  double dS[DIM], dL = 0.0;  // DER: S_d and sum_H a |G|^2 Re z
#pragma unroll
  for (int d = 0; d < DIM; ++d) dS[d] = 0.0;
  const R c2q = uniform_r(qk != 0.0 ? R(2.0 / qk) : R(0));
  const R qr = uniform_r(R(qk));
  for (int s = tid; s < nseg && (qk != 0.0 || acc); s += BLOCK) {
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
    double2 ro[SEG];  // the other plane's segment (layered system)
    if (lay)
#pragma unroll
      for (int j = 0; j < SEG; ++j) ro[j] = rhoo2[size_t(j) * nseg + s];
    if (acc) {  // the accepted move first, written back to its plane
      SegWalk<R> wpo(anchor<DIM, R>(tpo, pn, nm), upo, c2po), wpn(anchor<DIM, R>(tpn, pn, nm), upn, c2pn);
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const size_t g = size_t(j) * nseg + s;
        if (acc_own) {
          add_move(rcur[j], qp, wpn.cur, wpo.cur);
          rho2[g] = rcur[j];
        } else if (lay) {
          add_move(ro[j], qp, wpn.cur, wpo.cur);
          rhoo2[g] = ro[j];
        }
        if (j + 1 < SEG) {
          wpo.step(j);
          wpn.step(j);
        }
      }
    }
    SegWalk<R> wo(anchor<DIM, R>(to, pn, nm), uo, c2o), wn(anchor<DIM, R>(tn, pn, nm), un, c2n);
    float segE = 0.f, segJ = 0.f, segX = 0.f;  // mixed form: FP32 sums per segment, compensated across segments
    R sT = R(0), sT2 = R(0), sL = R(0);  // DER: per-segment sums of a Im z, j a Im z, a |G|^2 Re z
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const cplx<R> eo = wo.cur, en = wn.cur;
      const size_t g = size_t(j) * nseg + s;
      R wg, aj, ag2 = R(0);
      if (wlds) {
        const WT2 wa = ltab[scur[j]];
        wg = wa.x;
        aj = wa.y;
        if (DER) ag2 = ltab2[scur[j]];
      } else {
        wg = R(wt[g]);
        aj = ja ? R(ja[g]) : R(0);
        if (DER) ag2 = R(S->jg2_tab[scur[j]]);
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
      if (lay) {  // other plane: w_x (rho_o . d)
        const R xo = fma(R(ro[j].x), dx, R(ro[j].y) * dy);
        if (MIXED)
          segX = fmaf(float(S->wx[g]), float(xo), segX);
        else
          accX64 = fma(S->wx[g], double(xo), accX64);
      }
      if (DER) {
        const R px = fma(qr, dx, R(rcur[j].x)), py = fma(qr, dy, R(rcur[j].y));  // rho'
        const R im = fma(px, en.y, -(py * en.x)), re = fma(px, en.x, py * en.y);
        const R ti = aj * im;
        sT += ti;
        sT2 = fma(R(j), ti, sT2);
        sL = fma(ag2, re, sL);
      }
      if (j + 1 < SEG) {
        wo.step(j);
        wn.step(j);
      }
    }
    if (MIXED) {
      accE32.add(segE);
      if (ja) accJ32.add(segJ);
      if (lay) accX32.add(segX);
    }
    if (DER) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) dS[d] = fma(double(sT), double(unpack_n(pn, d)), dS[d]);
      dS[DIM - 1] += double(sT2);
      dL += double(sL);
    }
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      rcur[j] = rnxt[j];
      scur[j] = snxt[j];
    }
  }
  // real space (the accepted particle at its new position)
  UOut<DIM> ut;
  const double er = real_move<DIM, MIXED, PD, BLOCK, UJ, UJ && DER>(sn, so, k, spos, S->mobile_q, n, S, &ut,
                                                                    acc ? pk : -1, sp);
  const double q2 = qk * qk;
  constexpr int NP = DER ? 3 + DIM : 2;         // energy, J, and the p-term derivative sums
  constexpr int NV = NP + (UJ && DER ? DIM + 1 : 0);  // and the u term's gradient (frame axes) and Laplacian
  static_assert(NV * (BLOCK / 64) <= RED_DELTA, "reduction area too small");
  double v[NV];
  v[0] = q2 * (MIXED ? accE32.value() : accE64) + qk * er;
  if (lay) v[0] += 2.0 * qk * (MIXED ? accX32.value() : accX64);
  v[1] = q2 * (MIXED ? accJ32.value() : accJ64) + (UJ ? ut.d : 0.0);
  if (DER) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) v[2 + d] = dS[d];
    v[NP - 1] = dL;
  }
  if (UJ && DER) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) v[NP + d] = ut.g[d];
    v[NV - 1] = ut.l;
  }
  block_sum<NV>(v, red);  // (its barriers also order every read of the header and positions before the writes below)
  if (tid == 0) {
    delta[w] = v[0];
    if (djas) djas[w] = v[1];
    if (DER) {
      double ug[DIM];  // u term gradient in Cartesian axes (its sums are in the lower-triangular frame's)
      if (UJ) frame_to_cart<DIM>(v + NP, S->El, ug);
#pragma unroll
      for (int e = 0; e < DIM; ++e) {
        double gx = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) gx = fma(v[2 + d], S->B[d * 3 + e], gx);
        jgrad[size_t(w) * DIM + e] = -2.0 * qk * gx + (UJ ? ug[e] : 0.0);
      }
      jlap[w] = -2.0 * qk * v[NP - 1] + 2.0 * q2 * S->jlap_c + (UJ ? v[NV - 1] : 0.0);
    }
    if (accept_prev) accept_header<DIM>(hdr, spos, pk, acc, sp, K);
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
  const int n = W.n_mobile, nseg = S->n_seg, nm = S->nm;
  const int tbl = 2 * nm + 1;
  char* st = state + W.state_off;
  WalkerHdr* hdr = reinterpret_cast<WalkerHdr*>(st);
  double* spos = reinterpret_cast<double*>(st + HDR_BYTES);
  double* rho = reinterpret_cast<double*>(st + HDR_BYTES + walker_pos_bytes(n, DIM));
  cplx<R>* to = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* tn = to + DIM * tbl;

  const int pk = hdr->pending_k;
  const bool acc = pk >= 0 && pk < n && accept[w] != 0;
  double so[DIM], sn[DIM] = {};
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
    // a layered system's second plane keeps its rho after the first's
    const bool l1 = DIM == 2 && S->n_layers > 1 && pk >= S->n0;
    accept_stream<DIM, R>(S, to, tn, rho + (l1 ? 2 * size_t(SEG) * nseg : 0), R(S->mobile_q[pk]));
  }
  if (tid == 0) accept_header<DIM>(hdr, spos, pk, acc, sn, S->refresh_every);
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
  // a layered system: each plane from its own particles and ions
  const int n_planes = (DIM == 2 && S->n_layers > 1) ? 2 : 1;
  for (int l = 0; l < n_planes; ++l) {  // uniform
    const int p0 = l == 0 ? 0 : S->n0, p1 = n_planes == 1 ? n : (l == 0 ? S->n0 : n);
    double* rl = rho + 2 * size_t(SEG) * nseg * l;
    cplx<double> acc[1][SEG];
    rebuild_rho<DIM, 1>(acc, an, chunk * BLOCK + tid, S, spos + size_t(p0) * DIM, S->mobile_q + p0, p1 - p0,
                        tabs, TILE_P, l == 0 ? S->rho_fix : S->rho_fix1);
    if (s < nseg) {
      double drift = 0.0;
#pragma unroll
      for (int j = 0; j < SEG; ++j) {
        const size_t g = size_t(j) * nseg + s;
        drift = fmax(drift, fmax(fabs(acc[0][j].x - rl[2 * g]), fabs(acc[0][j].y - rl[2 * g + 1])));
        rl[2 * g] = acc[0][j].x;
        rl[2 * g + 1] = acc[0][j].y;
      }
      for (int off = 32; off > 0; off >>= 1) drift = fmax(drift, __shfl_xor(drift, off, 64));
      if ((tid & 63) == 0)
        atomicMax(reinterpret_cast<unsigned long long*>(&hdr->drift_max),
                  static_cast<unsigned long long>(__double_as_longlong(drift)));
    }
  }
  if (chunk == 0 && tid == 0) hdr->n_refresh += 1;
}

// ---------------------------------------------------------------------------
// launchers

namespace {

template <int DIM, int SPT, int PD, bool ORTHO, bool UJ>
int energy_inst(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
                void* stream) {
  const int lds_pos = even(b.max_particles);
  const size_t rpart = size_t(DIM) * (2 * b.max_nm + 1) * sizeof(cplx<double>);
  const size_t head = 16 * 8, pairs = size_t(lds_pos) * (DIM + 1) * 8;
  auto* kern = k_energy<DIM, SPT, PD, ORTHO, UJ>;
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

template <int DIM, int PD, bool ORTHO, bool UJ>
int energy_spt(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
               void* stream) {
  switch (spt_for(b.max_n_seg)) {
    case 1: return energy_inst<DIM, 1, PD, ORTHO, UJ>(b, pos, state, energy, jastrow, stream);
    case 2: return energy_inst<DIM, 2, PD, ORTHO, UJ>(b, pos, state, energy, jastrow, stream);
    case 4: return energy_inst<DIM, 4, PD, ORTHO, UJ>(b, pos, state, energy, jastrow, stream);
    default: return energy_inst<DIM, 8, PD, ORTHO, UJ>(b, pos, state, energy, jastrow, stream);
  }
}

template <int DIM, int PD, bool ORTHO>
int energy_pd(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
              void* stream) {
  return b.has_u ? energy_spt<DIM, PD, ORTHO, true>(b, pos, state, energy, jastrow, stream)
                 : energy_spt<DIM, PD, ORTHO, false>(b, pos, state, energy, jastrow, stream);
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
              double* djas, double* jgrad, double* jlap, void* stream, const uint8_t* accept_prev = nullptr,
              int redo = 0) {
  using R = typename std::conditional<MIXED, float, double>::type;
  // phase tables of the proposed move and of the accepted one (step form)
  const size_t mtab = size_t(4) * DIM * (2 * b.max_nm + 1) * sizeof(cplx<R>);
  const int lds_tab = even(int((mtab + 7) / 8));  // in doubles
  const bool der = jgrad != nullptr;
  const size_t lds = RED_DELTA * 8 + size_t(lds_tab) * 8 + size_t(b.max_wtab) * (sizeof(cplx<R>) + (der ? sizeof(R) : 0));
#define EW_DELTA(PD, DER, UJ)                                                                                     \
  hipLaunchKernelGGL((k_delta<DIM, MIXED, PD, DER, UJ>), dim3(b.n_walkers), dim3(BLOCK), lds, as_stream(stream), \
                     b.d_sys, b.d_walk, state, k, new_pos, delta, djas, jgrad, jlap, lds_tab, accept_prev, redo)
#define EW_DELTA_U(PD, DER) \
  if (b.has_u)              \
    EW_DELTA(PD, DER, true); \
  else                      \
    EW_DELTA(PD, DER, false)
  if (b.poly_deg <= 16) {
    if (der) {
      EW_DELTA_U(16, true);
    } else {
      EW_DELTA_U(16, false);
    }
  } else {
    if (der) {
      EW_DELTA_U(32, true);
    } else {
      EW_DELTA_U(32, false);
    }
  }
#undef EW_DELTA_U
#undef EW_DELTA
  return last_launch();
}

template <int DIM>
int rebuild_launch(const LaunchBatch& b, char* state, void* stream) {
  const size_t lds_r = size_t(TILE_P) * DIM * (2 * b.max_nm + 1) * sizeof(cplx<double>);
  const int chunks = (b.max_n_seg + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL((k_rebuild<DIM>), dim3(b.n_walkers, chunks), dim3(BLOCK), lds_r, as_stream(stream), b.d_sys,
                     b.d_walk, state);
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
  return rebuild_launch<DIM>(b, state, stream);
}

// Step: the previous move's accept folded into the new move's delta; in the
// FP32-mixed form the walkers whose accept reached the refresh count are
// rebuilt and their deltas recomputed from the rebuilt rho.
template <int DIM, bool MIXED>
int step_dim(const LaunchBatch& b, char* state, const uint8_t* accept_prev, const int32_t* k,
             const double* new_pos, double* delta, double* djas, double* jgrad, double* jlap, void* stream) {
  int rc = delta_dim<DIM, MIXED>(b, state, k, new_pos, delta, djas, jgrad, jlap, stream, accept_prev, 0);
  if (rc || !accept_prev || !MIXED || b.refresh_every <= 0) return rc;
  rc = rebuild_launch<DIM>(b, state, stream);
  if (rc) return rc;
  return delta_dim<DIM, MIXED>(b, state, k, new_pos, delta, djas, jgrad, jlap, stream, nullptr, 1);
}


int run_any(const LaunchBatch& b, const RunArgs& a) {
  if (!b.all_wtab_lds) return RUN_NO_FIT;
  const int jm = b.has_jastrow == 0 ? 0 : a.jgrad ? 2 : 1;
  if (b.has_u) {  // the u term comes with Jastrow outputs (JM 3, 4)
    if (b.dim == 3) {
      if (b.mixed) return jm == 2 ? run_d3_mixed_j4(b, a) : run_d3_mixed_j3(b, a);
      return jm == 2 ? run_d3_fp64_j4(b, a) : run_d3_fp64_j3(b, a);
    }
    if (b.mixed) return jm == 2 ? run_d2_mixed_j4(b, a) : run_d2_mixed_j3(b, a);
    return jm == 2 ? run_d2_fp64_j4(b, a) : run_d2_fp64_j3(b, a);
  }
  if (b.dim == 3) {
    if (b.mixed) return jm == 2 ? run_d3_mixed_j2(b, a) : jm ? run_d3_mixed_j1(b, a) : run_d3_mixed_j0(b, a);
    return jm == 2 ? run_d3_fp64_j2(b, a) : jm ? run_d3_fp64_j1(b, a) : run_d3_fp64_j0(b, a);
  }
  if (b.mixed) return jm == 2 ? run_d2_mixed_j2(b, a) : jm ? run_d2_mixed_j1(b, a) : run_d2_mixed_j0(b, a);
  return jm == 2 ? run_d2_fp64_j2(b, a) : jm ? run_d2_fp64_j1(b, a) : run_d2_fp64_j0(b, a);
}

}  // namespace

int launch_energy(const LaunchBatch& b, const double* pos, char* state, double* energy, double* jastrow,
                  void* stream) {
  return b.dim == 3 ? energy_dim<3>(b, pos, state, energy, jastrow, stream)
                   : energy_dim<2>(b, pos, state, energy, jastrow, stream);
}

int launch_delta(const LaunchBatch& b, char* state, const int32_t* k, const double* new_pos, double* delta,
                 double* djas, double* jgrad, double* jlap, void* stream) {
  if (b.dim == 3) return b.mixed ? delta_dim<3, true>(b, state, k, new_pos, delta, djas, jgrad, jlap, stream)
                                 : delta_dim<3, false>(b, state, k, new_pos, delta, djas, jgrad, jlap, stream);
  return b.mixed ? delta_dim<2, true>(b, state, k, new_pos, delta, djas, jgrad, jlap, stream)
                 : delta_dim<2, false>(b, state, k, new_pos, delta, djas, jgrad, jlap, stream);
}

int launch_step(const LaunchBatch& b, char* state, const uint8_t* accept_prev, const int32_t* k,
                const double* new_pos, double* delta, double* djas, double* jgrad, double* jlap, void* stream) {
  if (b.dim == 3)
    return b.mixed ? step_dim<3, true>(b, state, accept_prev, k, new_pos, delta, djas, jgrad, jlap, stream)
                   : step_dim<3, false>(b, state, accept_prev, k, new_pos, delta, djas, jgrad, jlap, stream);
  return b.mixed ? step_dim<2, true>(b, state, accept_prev, k, new_pos, delta, djas, jgrad, jlap, stream)
                 : step_dim<2, false>(b, state, accept_prev, k, new_pos, delta, djas, jgrad, jlap, stream);
}

int launch_accept(const LaunchBatch& b, char* state, const uint8_t* accept, void* stream) {
  if (b.dim == 3) return b.mixed ? accept_dim<3, true>(b, state, accept, stream) : accept_dim<3, false>(b, state, accept, stream);
  return b.mixed ? accept_dim<2, true>(b, state, accept, stream) : accept_dim<2, false>(b, state, accept, stream);
}

int launch_run(const LaunchBatch& b, char* state, int n_steps, const int32_t* k, const double* new_pos,
               const uint8_t* accept, double* delta, double* djas, double* jgrad, double* jlap, void* stream) {
  int rc = run_any(b, RunArgs{state, n_steps, k, new_pos, accept, delta, djas, jgrad, jlap, stream, nullptr});
  if (rc != RUN_NO_FIT) return rc;
  // a shell table or walker too large for LDS: the same sequence through the per-step kernels
  const size_t W = size_t(b.n_walkers);
  for (int m = 0; m < n_steps; ++m) {
    rc = launch_delta(b, state, k + m * W, new_pos + m * W * b.dim, delta + m * W, djas ? djas + m * W : nullptr,
                      jgrad ? jgrad + m * W * b.dim : nullptr, jlap ? jlap + m * W : nullptr, stream);
    if (!rc) rc = launch_accept(b, state, accept + m * W, stream);
    if (rc) return rc;
  }
  return 0;
}

void plan_run(const LaunchBatch& b, RunPlan* plan) {
  *plan = RunPlan{};
  if (run_any(b, RunArgs{nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, plan}) != 0)
    *plan = RunPlan{};
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
    (void)hipEventDestroy(e0);
    return int(hipErrorOutOfMemory);
  }
  int rc = launch_run(b, state, n_steps, k, new_pos, accept, delta, nullptr, nullptr, nullptr, stream);  // warm-up
  float best = 0.f;
  for (int r = 0; r < reps && !rc; ++r) {
    rc = int(hipEventRecord(e0, as_stream(stream)));
    if (!rc) rc = launch_run(b, state, n_steps, k, new_pos, accept, delta, nullptr, nullptr, nullptr, stream);
    if (!rc) rc = int(hipEventRecord(e1, as_stream(stream)));
    if (!rc) rc = int(hipEventSynchronize(e1));
    float ms = 0.f;
    if (!rc) rc = int(hipEventElapsedTime(&ms, e0, e1));
    if (!rc && (r == 0 || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  return rc;
}

int event_pair_create(void** pair) {
  hipEvent_t* e = new (std::nothrow) hipEvent_t[2];
  if (!e) return int(hipErrorOutOfMemory);
  hipError_t r = hipEventCreate(&e[0]);
  if (r == hipSuccess) {
    r = hipEventCreate(&e[1]);
    if (r != hipSuccess) (void)hipEventDestroy(e[0]);
  }
  if (r != hipSuccess) {
    delete[] e;
    return int(r);
  }
  *pair = e;
  return 0;
}

int event_pair_record(void* pair, int which, void* stream) {
  return int(hipEventRecord(static_cast<hipEvent_t*>(pair)[which], as_stream(stream)));
}

int event_pair_elapsed(void* pair, float* ms) {
  hipEvent_t* e = static_cast<hipEvent_t*>(pair);
  hipError_t r = hipEventSynchronize(e[1]);
  if (r == hipSuccess) r = hipEventElapsedTime(ms, e[0], e[1]);
  return int(r);
}

void event_pair_destroy(void* pair) {
  hipEvent_t* e = static_cast<hipEvent_t*>(pair);
  (void)hipEventDestroy(e[0]);
  (void)hipEventDestroy(e[1]);
  delete[] e;
}

int stream_capturing(void* stream, int* capturing) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  hipError_t r = hipStreamIsCapturing(as_stream(stream), &st);
  *capturing = st != hipStreamCaptureStatusNone;
  return int(r);
}

int stream_sync(void* stream) {
  hipError_t e = hipStreamSynchronize(as_stream(stream));
  return e == hipSuccess ? 0 : int(e);
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
int dev_cu_count(int* n_cu) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, dev);
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
