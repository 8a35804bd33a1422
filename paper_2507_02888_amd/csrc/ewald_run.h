// The fused multi-move kernel of libewald (gfx950) and its launch-shape
// templates.  Each (dimension, precision form, Jastrow) combination is
// instantiated in a translation unit of its own (ewald_run_d*.hip), so that
// the kernels compile in parallel.  Internal; not part of the public ABI.
#pragma once

#include "ewald_common.h"

namespace ewald {

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
  uint32_t wtab2, part2;  // Jastrow derivatives: a |G|^2 per shell, and the per-move partial sums
  uint32_t rcopy;  // 0, or the LDS copy of the running rho during a rebuild
  uint32_t next;   // queue mode: the next walker's index, broadcast to the workgroup
  int ch;     // moves per chunk
  int rtile;  // particles per rebuild tile (the tiles reuse the chunk tables)
};

// At least two waves per SIMD for workgroups of up to 512 threads (the
// register budget stays within 256 per lane; without the bound the compiler
// may take accumulation registers as well, which leaves one wave per SIMD).
// WV: the waves per SIMD a 256-thread kernel is bounded to (2, 3 or 4; 512 /
// WV registers per lane): small walkers may run more workgroups per CU with
// the pair-potential constants in scalar registers (WV > 2) than with them
// in vector registers (WV = 2); which wins depends on the batch, so the
// autotuner measures it.
// JM: Jastrow mode, 0 = none, 1 = J and dJ, 2 = also the gradient and the
// Laplacian of J with respect to the moved particle at each proposed
// configuration (as in k_delta: accumulated as S_d = sum_H a n_d Im z and
// sum_H a |G|^2 Re z, z = conj(rho') e'); 3 and 4 = 1 and 2 with the
// two-body polynomial term u of the mobile pairs added (its gradient summed
// in the geometry's frame axes, turned Cartesian once per move).
// LAY: layered 2D systems (two planes, no Jastrow terms): the second
// plane's rho in registers too, the cross-plane term 2 q sum_H w_x (rho_o . d)
// with w_x in the shell table's second column, real-space partners in the
// other plane sqrt(r^2 + dz^2) apart.  Walkers of a one-plane system run in
// such a kernel with an empty second plane.
// QUEUE = false: one walker per workgroup (walkers[blockIdx.x]; queue is
// unused).  QUEUE = true: `queue` is a work counter (zeroed before the
// launch) from which each workgroup takes the next walker index until all
// are done, in the launch order of `walkers` (most expensive first), so
// fewer workgroups than walkers serve the batch.  (A separate instantiation:
// the loop over walkers costs the one-walker kernels registers.)
template <int DIM, bool MIXED, int NT, int SPT, int PPR, int JM, int PD, bool ORTHO, bool XTRA, int WV = 2,
          bool LAY = false, bool QUEUE = false>
__global__ __launch_bounds__(NT, NT >= 1024 ? 4 : WV) void k_run(const DevSys* __restrict__ systems,
                                            const DevWalker* __restrict__ walkers, char* __restrict__ state,
                                            int n_steps, int n_walkers, const int32_t* __restrict__ kk,
                                            const double* __restrict__ new_pos, const uint8_t* __restrict__ accept,
                                            double* __restrict__ delta, double* __restrict__ djas,
                                            double* __restrict__ jgrad, double* __restrict__ jlap, RunLds L,
                                            int* __restrict__ queue) {
  constexpr bool JAS = JM > 0, DER = JM == 2 || JM == 4, UJ = JM >= 3;
  constexpr int NDP = DIM + 1;               // p-term derivative sums per move: S_0 .. S_{DIM-1}, L
  constexpr int NDV = UJ ? 2 * NDP : NDP;    // plus the u term's gradient (frame axes) and Laplacian
  using R = typename std::conditional<MIXED, float, double>::type;
  using WT = R;          // the mixed form multiplies weights with FP32 terms
  using WT2 = cplx<WT>;  // (weight, Jastrow coefficient)
  constexpr int NW = NT / 64;
  // PPR: own particles per thread held in registers (particles j = t + c NT, c < PPR)
  extern __shared__ __align__(16) char lds[];
  for (int wi = blockIdx.x;;) {
  if (QUEUE) {
    int* st_next = reinterpret_cast<int*>(lds + L.next);
    if (threadIdx.x == 0) *st_next = atomicAdd(queue, 1);
    __syncthreads();
    wi = uniform_i(*st_next);  // the walker is the same for every lane: its fields stay scalar
    __syncthreads();          // every thread has read the index before it is replaced
    if (wi >= n_walkers) break;
  }
  const DevWalker W = walkers[wi];
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
  double* st_part2 = reinterpret_cast<double*>(lds + L.part2);  // DER: [CH][NW][4 rows][NDV]
  WT* ltab2 = reinterpret_cast<WT*>(lds + L.wtab2);              // DER: a |G|^2 per shell
  int* st_k = reinterpret_cast<int*>(lds + L.k);
  int* st_acc = reinterpret_cast<int*>(lds + L.acc);
  int* st_cnt = reinterpret_cast<int*>(lds + L.cnt);

  for (int i = tid; i < n * DIM; i += NT) lpos[i] = spos[i];
  for (int i = tid; i < n; i += NT) lq[i] = S->mobile_q[i];
  // every system of the batch has its shell table in LDS (checked by the launcher)
  for (int i = tid; i < S->n_wtab; i += NT) {
    ltab[i] = {WT(S->wa_tab[2 * i]), WT(LAY ? (S->wx_tab ? S->wx_tab[i] : 0.0) : S->wa_tab[2 * i + 1])};
    if (DER) ltab2[i] = WT(S->jg2_tab[i]);
  }
  const bool lay = LAY && S->n_layers > 1;  // uniform
  const int n0 = LAY ? S->n0 : n;
  double* rho1 = rho + 2 * size_t(SEG) * nseg;  // the second plane (LAY)
  int counter = hdr->counter;
  int n_acc = hdr->n_accepts, n_ref = hdr->n_refresh;
  double drift = hdr->drift_max;
  if (K > 0 && counter >= K) counter = 0;

  double ps[PPR][DIM], pq[PPR];
  int psp[PPR];  // UJ: spin labels of the thread's own particles
#pragma unroll
  for (int c = 0; c < PPR; ++c) {
    const int j = tid + c * NT;
    double sj[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) sj[d] = j < n ? spos[j * DIM + d] : 0.0;
    geo_pos<DIM, ORTHO>(sj, S, ps[c]);
    pq[c] = j < n ? S->mobile_q[j] : 0.0;
    psp[c] = (UJ && j < n) ? S->spin[j] : 0;
  }
  // Workgroups of up to 512 threads (256 vector registers per lane) hold the
  // pair-polynomial coefficients in vector registers for the whole sweep
  // (loaded with a lane-varying index, so they are not taken for scalars);
  // that leaves the scalar registers to the loop state, which otherwise
  // spills into vector-register lanes.  With 1024 threads they stay scalar.
  constexpr int PF = PD == 16 ? 12 : 22;
  constexpr bool CV = NT <= 512 && WV <= 2;
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
  cplx<double> rv2[LAY ? SPT : 1][SEG];  // LAY: the second plane
  uint32_t shp[SPT][SEG / 2];  // two 16-bit shell-table byte offsets per register
#pragma unroll
  for (int i = 0; i < SPT; ++i) {
    const int s = tid + i * NT;
    an[i] = s < nseg ? S->seg_n[s] : 0u;
#pragma unroll
    for (int j = 0; j < SEG; ++j) {
      const size_t g = size_t(j) * nseg + s;
      rv[i][j] = s < nseg ? cplx<double>{rho[2 * g], rho[2 * g + 1]} : cplx<double>{0.0, 0.0};
      if constexpr (LAY)
        rv2[i][j] = (lay && s < nseg) ? cplx<double>{rho1[2 * g], rho1[2 * g + 1]} : cplx<double>{0.0, 0.0};
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
      const int k = uniform_i(st_k[mm]);  // the move's index, decision and charge are uniform
      double v0 = 0.0, v1 = 0.0;
      double dv[DER ? NDV : 1];  // DER: this thread's S_d and a |G|^2 Re z sums
#pragma unroll
      for (int d = 0; d < (DER ? NDV : 1); ++d) dv[d] = 0.0;
      if (k >= 0) {  // uniform
        const bool acc = uniform_i(st_acc[mm]) != 0;
        const double qk = uniform_d(lq[k]);
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
          const R q = R(qk), c2q = R(uniform_d(st_c2q[mm]));
          const R qa = acc ? q : R(0);
          double accE64 = 0.0, accJ64 = 0.0, accX64 = 0.0;
          Kahan accE32, accJ32, accX32;  // mixed form: FP32 sums per segment, compensated across segments
          if constexpr (LAY) {
            // own plane own[], other plane oth[]: the term as below plus the
            // cross-plane sum w_x (rho_o . d); one copy of the loop per plane
            // of the moved particle (uniform), so no per-lane selects
            auto lay_loop = [&](auto own2) {
              constexpr bool O2 = decltype(own2)::value;
              auto& own = pick_ref<O2>(rv, rv2);
              auto& oth = pick_ref<!O2>(rv, rv2);
#pragma unroll
              for (int i = 0; i < SPT; ++i) {
                if (tid + i * NT < nseg) {
                  SegWalk<R> wo(anchor<DIM, R>(to, an[i], nm), uo), wn(anchor<DIM, R>(tn, an[i], nm), un);
                  float segE = 0.f, segX = 0.f;
#pragma unroll
                  for (int j = 0; j < SEG; ++j) {
                    const cplx<R> eo = wo.cur, en = wn.cur;
                    const uint32_t off = (shp[i][j >> 1] >> (16 * (j & 1))) & 0xffffu;
                    const WT2 wa = ld_at_byte(ltab, off);  // (w, w_x)
                    const R dx = en.x - eo.x, dy = en.y - eo.y;
                    const R ux = fma(c2q, R(own[i][j].x), dx), uy = fma(c2q, R(own[i][j].y), dy);
                    const R t = fma(ux, dx, uy * dy);
                    const R xo = fma(R(oth[i][j].x), dx, R(oth[i][j].y) * dy);
                    if (MIXED) {
                      segE = fmaf(float(wa.x), float(t), segE);
                      segX = fmaf(float(wa.y), float(xo), segX);
                    } else {
                      accE64 = fma(double(wa.x), double(t), accE64);
                      accX64 = fma(double(wa.y), double(xo), accX64);
                    }
                    own[i][j].x += double(qa * dx);
                    own[i][j].y += double(qa * dy);
                    if (j + 1 < SEG) {
                      wo.step(j);
                      wn.step(j);
                    }
                  }
                  if (MIXED) {
                    accE32.add(segE);
                    accX32.add(segX);
                  }
                }
              }
            };
            if (k >= n0)
              lay_loop(std::true_type{});
            else
              lay_loop(std::false_type{});
          } else {
#pragma unroll
          for (int i = 0; i < SPT; ++i) {
            if (tid + i * NT < nseg) {
              SegWalk<R> wo(anchor<DIM, R>(to, an[i], nm), uo), wn(anchor<DIM, R>(tn, an[i], nm), un);
              float segE = 0.f, segJ = 0.f;
              R sT = R(0), sT2 = R(0), sL = R(0);  // DER: sums of a Im z, j a Im z, a |G|^2 Re z
#pragma unroll
              for (int j = 0; j < SEG; ++j) {
                const cplx<R> eo = wo.cur, en = wn.cur;
                const uint32_t off = (shp[i][j >> 1] >> (16 * (j & 1))) & 0xffffu;
                const WT2 wa = ld_at_byte(ltab, off);
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
                if (DER) {
                  const WT ag2 = *reinterpret_cast<const WT*>(reinterpret_cast<const char*>(ltab2) + (off >> 1));
                  const R px = fma(q, dx, R(rv[i][j].x)), py = fma(q, dy, R(rv[i][j].y));  // rho'
                  const R im = fma(px, en.y, -(py * en.x)), re = fma(px, en.x, py * en.y);
                  const R ti = R(wa.y) * im;
                  sT += ti;
                  sT2 = fma(R(j), ti, sT2);
                  sL = fma(R(ag2), re, sL);
                }
                // rho += q d on an accepted move: the charge times the uniform
                // decision (0 when rejected, which adds an exact zero) instead
                // of a branch the compiler would turn into per-lane selects
                rv[i][j].x += double(qa * dx);
                rv[i][j].y += double(qa * dy);
                if (j + 1 < SEG) {
                  wo.step(j);
                  wn.step(j);
                }
              }
              if (MIXED) {
                accE32.add(segE);
                if (JAS) accJ32.add(segJ);
              }
              if (DER) {
#pragma unroll
                for (int d = 0; d < DIM; ++d) dv[d] = fma(double(sT), double(unpack_n(an[i], d)), dv[d]);
                dv[DIM - 1] += double(sT2);
                dv[DIM] += double(sL);
              }
            }
          }
          }
          const double q2 = qk * qk;
          v0 = q2 * (MIXED ? accE32.value() : accE64);
          if (LAY) v0 += 2.0 * qk * (MIXED ? accX32.value() : accX64);
          if (JAS) v1 = q2 * (MIXED ? accJ32.value() : accJ64);
          if (!UJ)
            v0 += qk * real_move_own<DIM, MIXED, PD, NT, PPR, ORTHO, XTRA, false, false, LAY>(
                           xn, xo, k, ps, pq, lpos, lq, n, S, c64, c32, CV ? fk : frame_k(S), nullptr, 0, nullptr,
                           lay, n0, LAY ? S->dz2 : 0.0);
        }
        if (UJ) {  // the u term moves with a neutral particle too
          UOut<DIM> uo;
          const double er = real_move_own<DIM, MIXED, PD, NT, PPR, ORTHO, XTRA, UJ, DER>(
              xn, xo, k, ps, pq, lpos, lq, n, S, c64, c32, CV ? fk : frame_k(S), psp, S->spin[k], &uo);
          v0 += qk * er;
          v1 += uo.d;
          if (DER) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) dv[NDP + d] = uo.g[d];
            dv[NDV - 1] = uo.l;
          }
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
      if (DER)
#pragma unroll
        for (int d = 0; d < NDV; ++d) dv[d] = row_sum16(dv[d]);
      if ((lane & 15) == 0) {
        double* p = st_part + ((mm * NW + wave) * 4 + (lane >> 4)) * 2;
        p[0] = v0;
        p[1] = v1;
        if (DER) {
          double* p2 = st_part2 + ((mm * NW + wave) * 4 + (lane >> 4)) * NDV;
#pragma unroll
          for (int d = 0; d < NDV; ++d) p2[d] = dv[d];
        }
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
      if (DER) {
        const int kq = st_k[tid];
        double sv[NDV];
#pragma unroll
        for (int d = 0; d < NDV; ++d) sv[d] = 0.0;
        if (kq >= 0) {
          const double* p2 = st_part2 + tid * NW * 4 * NDV;
          for (int v = 0; v < NW * 4; ++v)
#pragma unroll
            for (int d = 0; d < NDV; ++d) sv[d] += p2[v * NDV + d];
        }
        const double qk = kq >= 0 ? lq[kq] : 0.0;
        double ug[DIM];  // u term gradient in Cartesian axes
        if (UJ) frame_to_cart<DIM>(sv + NDP, ORTHO ? S->Eo : S->El, ug);
#pragma unroll
        for (int e2 = 0; e2 < DIM; ++e2) {
          double gx = 0.0;
#pragma unroll
          for (int d = 0; d < DIM; ++d) gx = fma(sv[d], S->B[d * 3 + e2], gx);
          jgrad[idx * DIM + e2] = kq < 0 ? NAN : -2.0 * qk * gx + (UJ ? ug[e2] : 0.0);
        }
        jlap[idx] = kq < 0 ? NAN : -2.0 * qk * sv[DIM] + 2.0 * qk * qk * S->jlap_c + (UJ ? sv[NDV - 1] : 0.0);
      }
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
      if constexpr (LAY) {
        // a layered walker: the second plane's running rho kept in its state
        // block, each plane rebuilt from its own particles and ions
        if (lay) {
#pragma unroll
          for (int i = 0; i < SPT; ++i) {
            const int s = tid + i * NT;
            if (s < nseg)
#pragma unroll
              for (int j = 0; j < SEG; ++j) {
                const size_t g = size_t(j) * nseg + s;
                rho1[2 * g] = rv2[i][j].x;
                rho1[2 * g + 1] = rv2[i][j].y;
              }
          }
          rebuild_rho<DIM, SPT, NT>(rv2, an, tid, S, lpos + size_t(n0) * DIM, lq + n0, n - n0, tabs, L.rtile,
                                    S->rho_fix1);
        }
      }
      rebuild_rho<DIM, SPT, NT>(rv, an, tid, S, lpos, lq, n0, tabs, L.rtile);
      double dm = 0.0;
      if constexpr (LAY) {
        if (lay) {
#pragma unroll
          for (int i = 0; i < SPT; ++i) {
            const int s = tid + i * NT;
            if (s < nseg)
#pragma unroll
              for (int j = 0; j < SEG; ++j) {
                const size_t g = size_t(j) * nseg + s;
                dm = fmax(dm, fmax(fabs(rv2[i][j].x - rho1[2 * g]), fabs(rv2[i][j].y - rho1[2 * g + 1])));
              }
          }
        }
      }
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
        if constexpr (LAY) {
          if (lay) {
            rho1[2 * g] = rv2[i][j].x;
            rho1[2 * g + 1] = rv2[i][j].y;
          }
        }
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
  if (!QUEUE) break;
  __syncthreads();  // the next walker reuses LDS
  }
}

// The fused kernel's work counter, zeroed on the stream before a queue-mode
// launch (a kernel rather than a memset, so that graph capture records it
// as a kernel node).
template <int D>
__global__ void k_queue_reset(int* queue) {
  if (threadIdx.x == 0) *queue = 0;
}

// ---------------------------------------------------------------------------
// launch shapes


// LDS layout of the fused kernel for a chunk of ch moves; returns the total bytes.
template <int DIM, bool MIXED, int NT, int SPT, bool DER, bool UJ = false>
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
  // DER: a |G|^2 per shell, read by every move of the sweep, so it sits
  // before the region that the rebuild between chunks reuses
  L.wtab2 = 0;
  if (DER) {
    L.wtab2 = uint32_t(o);
    o = up16(o + size_t(b.max_wtab) * sizeof(R));
  }
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
  L.next = uint32_t(o);
  o = up16(o + 4);
  L.part2 = 0;
  if (DER) {
    L.part2 = uint32_t(o);
    o = up16(o + size_t(ch) * NW * 4 * (DIM + 1) * (UJ ? 2 : 1) * 8);
  }
  L.ch = ch;
  // between chunks everything from ctab on holds per-chunk data only, so the
  // rebuild tiles may fill all of it; even (the tiles interleave particle pairs)
  L.rtile = int(std::min<size_t>((o - L.ctab) / rpart, 64)) & ~1;
  // Between chunks the tables and the staging area (everything from ctab on:
  // per-chunk data only) are free: the mixed form's rebuild keeps the running
  // rho there (for the drift check) when it fits beside tiles of at least
  // TILE_P particles, instead of a round trip through HBM.
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
  double* jgrad;  // non-null (with jlap): Jastrow derivatives per move
  double* jlap;
  void* stream;
  RunPlan* plan;  // non-null: resolve the launch shape only, launch nothing
};

template <int DIM, bool MIXED, int NT, int SPT, int PPR, int JM, int PD, bool ORTHO, bool XTRA, int WV = 2,
          bool LAY = false, bool QUEUE = false>
int run_inst(const LaunchBatch& b, const RunArgs& a) {
  auto* kern = k_run<DIM, MIXED, NT, SPT, PPR, JM, PD, ORTHO, XTRA, WV, LAY, QUEUE>;
  constexpr bool DER = JM == 2 || JM == 4, UJ = JM >= 3;
  static const int per_cu = blocks_per_cu(kern, NT);
  const size_t budget = RUN_LDS_BUDGET / size_t(per_cu);
  RunLds L{};
  int ch = b.run_chunk > 0 ? std::min(b.run_chunk, RUN_CHUNK) : RUN_CHUNK;
  size_t lds = run_layout<DIM, MIXED, NT, SPT, DER, UJ>(b, ch, L);
  if (b.run_chunk <= 0)
    while (lds > budget && ch > 8) lds = run_layout<DIM, MIXED, NT, SPT, DER, UJ>(b, --ch, L);
  while (lds > RUN_LDS_BUDGET && ch > 1) lds = run_layout<DIM, MIXED, NT, SPT, DER, UJ>(b, --ch, L);
  if (lds > RUN_LDS_BUDGET) return RUN_NO_FIT;
  // queue mode: ceil(W / walkers_per_block) workgroups take walkers from a
  // counter in the state buffer
  const int wpb = QUEUE ? b.run_wpb : 0;
  const int grid = wpb > 0 ? (b.n_walkers + wpb - 1) / wpb : b.n_walkers;
  if (a.plan) {
    *a.plan = RunPlan{1, NT, SPT, PPR, ch, ORTHO ? 0 : 1, int(lds), per_cu, NT <= 512 ? WV : 0, wpb, grid};
    return 0;
  }
  if (int rc = allow_lds(kern, lds)) return rc;
  int* queue = nullptr;
  if (QUEUE) {
    queue = reinterpret_cast<int*>(a.state + QUEUE_OFF);
    hipLaunchKernelGGL(k_queue_reset<0>, dim3(1), dim3(64), 0, as_stream(a.stream), queue);
    if (int rc = last_launch()) return rc;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, as_stream(a.stream), b.d_sys, b.d_walk, a.state,
                     a.n_steps, b.n_walkers, a.k, a.new_pos, a.accept, a.delta, a.djas, a.jgrad, a.jlap, L, queue);
  return last_launch();
}

// Workgroup shapes of the fused kernel (threads NT, segments per thread SPT).
// A shape is available for a batch when NT SPT covers its largest segment
// count s and no smaller SPT would (so each NT appears once); `threads`
// picks among the available ones, 0 = the default (the first listed that is
// available):
//   s <= 256: 256 x 1          s <= 512: 256 x 2
//   s <= 1024: 1024 x 1, or 512 x 2      s <= 2048: 512 x 4
// (1024 x 1 is also available for s <= 512).  Workgroups sized to small
// walkers (320, 384 or 512 threads with one segment and one particle per
// lane) were measured slower than 256 x 2 on the 250-, 300- and uneven
// 64..512-electron workloads: at ~200 registers per lane such a kernel fits
// one workgroup per CU, where 256-thread ones fit two.
// Particles per thread in registers: 1 when the largest walker has at most
// NT particles (always with 1024 threads, where larger walkers' remaining
// particles are read from LDS), else 2.
inline int run_shape(int max_n_seg, int max_particles, int threads, int* nt, int* spt, int* ppr) {
  struct Shape { int nt, spt; };
  static const Shape shapes[] = {{256, 1}, {256, 2}, {1024, 1}, {512, 2}, {512, 4}};
  for (const Shape& sh : shapes) {
    if (sh.nt * sh.spt < max_n_seg) continue;                          // does not cover the segments
    if (sh.spt > 1 && sh.nt * (sh.spt / 2) >= max_n_seg) continue;    // a smaller SPT would
    if (threads == 0 || threads == sh.nt) {
      *nt = sh.nt;
      *spt = sh.spt;
      *ppr = (sh.nt >= 1024 || max_particles <= sh.nt) ? 1 : 2;
      return 1;
    }
  }
  return 0;
}

template <int DIM, bool MIXED, int JM, int PD, bool ORTHO, bool LAY = false>
int run_jp(const LaunchBatch& b, const RunArgs& a) {
  static_assert(RUN_CHUNK <= 256, "staging uses one thread per move");
  int nt = 0, spt = 0, ppr = 0;
  if (!run_shape(b.max_n_seg, b.max_particles, b.run_threads, &nt, &spt, &ppr)) return RUN_NO_FIT;
  // XTRA: particles beyond the registers' share, or fixed ions, in some
  // walker.  Leaving those loops out pays at 512 and 1024 threads; the
  // 256-thread kernels keep them (without them the compiler spends more
  // registers there and runs slower).
  const bool xtra = b.max_particles > ppr * nt || b.max_fixed > 0;
  const int wv = b.run_waves > 0 ? b.run_waves : 2;
  // the queue mode is compiled for two waves per SIMD; the host rejects it
  // with other wave counts
  const bool queue = b.run_wpb > 0;
#define EW_RUN(NT, SPT, PPR)                                                                             \
  if (nt == NT && spt == SPT && ppr == PPR) {                                                           \
    if (wv == 3) return run_inst<DIM, MIXED, NT, SPT, PPR, JM, PD, ORTHO, true, 3, LAY>(b, a);          \
    if (wv == 4) return run_inst<DIM, MIXED, NT, SPT, PPR, JM, PD, ORTHO, true, 4, LAY>(b, a);          \
    return queue ? run_inst<DIM, MIXED, NT, SPT, PPR, JM, PD, ORTHO, true, 2, LAY, true>(b, a)          \
                 : run_inst<DIM, MIXED, NT, SPT, PPR, JM, PD, ORTHO, true, 2, LAY>(b, a);               \
  }
#define EW_RUN_X(NT, SPT, PPR)                                                                          \
  if (nt == NT && spt == SPT && ppr == PPR)                                                            \
    return queue ? (xtra ? run_inst<DIM, MIXED, NT, SPT, PPR, JM, PD, ORTHO, true, 2, LAY, true>(b, a)   \
                         : run_inst<DIM, MIXED, NT, SPT, PPR, JM, PD, ORTHO, false, 2, LAY, true>(b, a)) \
                 : (xtra ? run_inst<DIM, MIXED, NT, SPT, PPR, JM, PD, ORTHO, true, 2, LAY>(b, a)         \
                         : run_inst<DIM, MIXED, NT, SPT, PPR, JM, PD, ORTHO, false, 2, LAY>(b, a))
  EW_RUN(256, 1, 1);
  EW_RUN(256, 1, 2);
  EW_RUN(256, 2, 1);
  EW_RUN(256, 2, 2);
  EW_RUN_X(1024, 1, 1);
  // 512 x 2 also at four waves per SIMD (two workgroups per CU, 128
  // registers): faster for the FP32-mixed form, slower for FP64.  The
  // Jastrow-derivative kernels (JM 2, 4) need more registers: they stay at
  // two waves whatever the tuning says (the autotuner probes without them).
  constexpr bool DERJ = JM == 2 || JM == 4;
  if (!DERJ && nt == 512 && spt == 2 && ppr == 2 && wv == 4 && !queue)
    return xtra ? run_inst<DIM, MIXED, 512, 2, 2, JM, PD, ORTHO, true, 4, LAY>(b, a)
                : run_inst<DIM, MIXED, 512, 2, 2, JM, PD, ORTHO, false, 4, LAY>(b, a);
  EW_RUN_X(512, 2, 2);
  EW_RUN_X(512, 4, 2);
#undef EW_RUN_X
#undef EW_RUN
  return RUN_NO_FIT;
}

template <int DIM, bool MIXED, int JM, int PD>
int run_jpo(const LaunchBatch& b, const RunArgs& a) {
  // layered 2D batches (no Jastrow terms) take the kernels with a second plane
  if constexpr (DIM == 2 && JM == 0) {
    if (b.layered)
      return b.all_ortho && !b.general_frame ? run_jp<DIM, MIXED, JM, PD, true, true>(b, a)
                                             : run_jp<DIM, MIXED, JM, PD, false, true>(b, a);
  }
  return b.all_ortho && !b.general_frame ? run_jp<DIM, MIXED, JM, PD, true>(b, a)
                                         : run_jp<DIM, MIXED, JM, PD, false>(b, a);
}


template <int DIM, bool MIXED, int JM>
int run_entry(const LaunchBatch& b, const RunArgs& a) {
  return b.poly_deg <= 16 ? run_jpo<DIM, MIXED, JM, 16>(b, a) : run_jpo<DIM, MIXED, JM, 32>(b, a);
}

// One per translation unit: run_entry<DIM, MIXED, JM> (JM = Jastrow mode).
int run_d3_fp64_j0(const LaunchBatch& b, const RunArgs& a);
int run_d3_fp64_j1(const LaunchBatch& b, const RunArgs& a);
int run_d3_fp64_j2(const LaunchBatch& b, const RunArgs& a);
int run_d3_mixed_j0(const LaunchBatch& b, const RunArgs& a);
int run_d3_mixed_j1(const LaunchBatch& b, const RunArgs& a);
int run_d3_mixed_j2(const LaunchBatch& b, const RunArgs& a);
int run_d2_fp64_j0(const LaunchBatch& b, const RunArgs& a);
int run_d2_fp64_j1(const LaunchBatch& b, const RunArgs& a);
int run_d2_fp64_j2(const LaunchBatch& b, const RunArgs& a);
int run_d2_mixed_j0(const LaunchBatch& b, const RunArgs& a);
int run_d2_mixed_j1(const LaunchBatch& b, const RunArgs& a);
int run_d2_mixed_j2(const LaunchBatch& b, const RunArgs& a);
// the same with the Jastrow u term (JM = 3: J and dJ; 4: also derivatives)
int run_d3_fp64_j3(const LaunchBatch& b, const RunArgs& a);
int run_d3_fp64_j4(const LaunchBatch& b, const RunArgs& a);
int run_d3_mixed_j3(const LaunchBatch& b, const RunArgs& a);
int run_d3_mixed_j4(const LaunchBatch& b, const RunArgs& a);
int run_d2_fp64_j3(const LaunchBatch& b, const RunArgs& a);
int run_d2_fp64_j4(const LaunchBatch& b, const RunArgs& a);
int run_d2_mixed_j3(const LaunchBatch& b, const RunArgs& a);
int run_d2_mixed_j4(const LaunchBatch& b, const RunArgs& a);

}  // namespace ewald
