// Host side of libewald: argument validation, the FP64 set-up tables of a
// periodic cell (paper Sec. 2.2; Sec. 6.1 keeps these tables in double
// precision), walker-batch layout and the C ABI entry points.
//
// Nothing here touches a GPU until ewald_batch_create uploads the tables, so
// every validation path and every table can be checked on a machine without
// one.

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ewald.h"
#include "ewald_internal.h"

using namespace ewald;

namespace {

thread_local std::string g_last_error;

ewald_status fail(ewald_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

constexpr double kPi = 3.14159265358979323846;

}  // namespace

namespace ewald {
// the message for ewald_last_error, from the library's other translation units
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace ewald

namespace {

bool is_fin(double x) { return std::isfinite(x); }

// 3x3 helpers on row-major arrays; a 2D cell lives in the upper-left 2x2
// block with the rest zero.
double det_n(const double* a, int dim) {
  if (dim == 2) return a[0] * a[4] - a[1] * a[3];
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}

void inverse_n(const double* a, int dim, double* inv) {
  std::fill(inv, inv + 9, 0.0);
  double d = det_n(a, dim);
  if (dim == 2) {
    inv[0] = a[4] / d;
    inv[1] = -a[1] / d;
    inv[3] = -a[3] / d;
    inv[4] = a[0] / d;
    return;
  }
  inv[0] = (a[4] * a[8] - a[5] * a[7]) / d;
  inv[1] = (a[2] * a[7] - a[1] * a[8]) / d;
  inv[2] = (a[1] * a[5] - a[2] * a[4]) / d;
  inv[3] = (a[5] * a[6] - a[3] * a[8]) / d;
  inv[4] = (a[0] * a[8] - a[2] * a[6]) / d;
  inv[5] = (a[2] * a[3] - a[0] * a[5]) / d;
  inv[6] = (a[3] * a[7] - a[4] * a[6]) / d;
  inv[7] = (a[1] * a[6] - a[0] * a[7]) / d;
  inv[8] = (a[0] * a[4] - a[1] * a[3]) / d;
}

double wrap01(double x) {
  double f = x - std::floor(x);
  return f >= 1.0 ? 0.0 : f;
}

// Orthogonal sublattice of index 1 or 2 whose coset sits at half box sides
// (simple-cubic, bcc, fcc and hexagonal cells have one).  Integer vectors
// with coefficients in [-2, 2] are searched for dim mutually orthogonal
// lattice vectors v_d = n_d A of the smallest index |det n| <= 2; the coset of
// the sublattice they span is found by reducing lattice points into the box
// spanned by them, and accepted only if every component of its offset is 0
// or half the box side.  Returns false if no such frame exists (the kernels
// then use the general reduction with candidate images).
struct OrthoFrame {
  double F[9] = {0};    // x = s F (frame coordinates from fractional ones)
  double E[9] = {0};    // rows: the frame's axes as Cartesian unit vectors
  double box[3] = {0};
  int n_coset = 0;
  double cw[MAX_COSET][3] = {{0}};
  double cc[MAX_COSET] = {0};
};

bool ortho_frame(const double* A, int dim, OrthoFrame& out) {
  std::vector<std::array<int, 3>> ns;
  std::vector<std::array<double, 3>> vs;
  const int R = 2;
  for (int a = -R; a <= R; ++a)
    for (int b = -R; b <= R; ++b)
      for (int c = (dim == 3 ? -R : 0); c <= (dim == 3 ? R : 0); ++c) {
        const int n[3] = {a, b, c};
        int first = 0;
        for (int d = 0; d < dim && first == 0; ++d) first = n[d];
        if (first <= 0) continue;  // one of each +-pair, no zero vector
        std::array<double, 3> v = {0, 0, 0};
        for (int i = 0; i < dim; ++i)
          for (int x = 0; x < 3; ++x) v[x] += n[i] * A[i * 3 + x];
        ns.push_back({a, b, c});
        vs.push_back(v);
      }
  auto dot = [](const std::array<double, 3>& u, const std::array<double, 3>& v) {
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
  };
  auto orth = [&](size_t i, size_t j) {
    return std::fabs(dot(vs[i], vs[j])) <= 1e-12 * std::sqrt(dot(vs[i], vs[i]) * dot(vs[j], vs[j]));
  };
  int best_index = 3;
  double best_len = INFINITY;
  size_t pick[3] = {0, 0, 0};
  const size_t nv = vs.size();
  for (size_t i = 0; i < nv; ++i)
    for (size_t j = i + 1; j < nv; ++j) {
      if (!orth(i, j)) continue;
      for (size_t k = (dim == 3 ? j + 1 : 0); k < (dim == 3 ? nv : 1); ++k) {
        if (dim == 3 && (!orth(i, k) || !orth(j, k))) continue;
        const auto &p = ns[i], &q = ns[j];
        int det;
        double len = std::sqrt(dot(vs[i], vs[i])) + std::sqrt(dot(vs[j], vs[j]));
        if (dim == 3) {
          const auto& r = ns[k];
          det = p[0] * (q[1] * r[2] - q[2] * r[1]) - p[1] * (q[0] * r[2] - q[2] * r[0]) +
                p[2] * (q[0] * r[1] - q[1] * r[0]);
          len += std::sqrt(dot(vs[k], vs[k]));
        } else {
          det = p[0] * q[1] - p[1] * q[0];
        }
        det = std::abs(det);
        if (det == 0 || det > best_index || (det == best_index && len >= best_len)) continue;
        best_index = det;
        best_len = len;
        pick[0] = i;
        pick[1] = j;
        pick[2] = k;
      }
    }
  if (best_index > 2) return false;
  double e[3][3] = {{0}};
  for (int d = 0; d < dim; ++d) {
    const auto& v = vs[pick[d]];
    out.box[d] = std::sqrt(dot(v, v));
    for (int x = 0; x < 3; ++x) e[d][x] = v[x] / out.box[d];
  }
  for (int i = 0; i < dim; ++i)
    for (int d = 0; d < dim; ++d)
      out.F[i * 3 + d] = A[i * 3] * e[d][0] + A[i * 3 + 1] * e[d][1] + A[i * 3 + 2] * e[d][2];
  for (int d = 0; d < 3; ++d)
    for (int x = 0; x < 3; ++x) out.E[d * 3 + x] = e[d][x];
  // cosets: lattice points k A, k in [0, index)^dim, reduced into the box
  std::vector<std::array<double, 3>> reps;
  const int m = best_index;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      for (int c = 0; c < (dim == 3 ? m : 1); ++c) {
        const int k[3] = {a, b, c};
        std::array<double, 3> x = {0, 0, 0};
        for (int d = 0; d < dim; ++d) {
          for (int i = 0; i < dim; ++i) x[d] += k[i] * out.F[i * 3 + d];
          x[d] -= out.box[d] * std::nearbyint(x[d] / out.box[d]);
          if (std::fabs(std::fabs(x[d]) - 0.5 * out.box[d]) <= 1e-9 * out.box[d]) x[d] = 0.5 * out.box[d];
          if (std::fabs(x[d]) <= 1e-9 * out.box[d]) x[d] = 0.0;
        }
        bool seen = false;
        for (const auto& r : reps) {
          bool same = true;
          for (int d = 0; d < dim; ++d) same = same && std::fabs(r[d] - x[d]) <= 1e-9 * out.box[d];
          seen = seen || same;
        }
        if (!seen) reps.push_back(x);
      }
  if (int(reps.size()) != m) return false;
  out.n_coset = 0;
  for (const auto& r : reps) {
    bool zero = true;
    for (int d = 0; d < dim; ++d) zero = zero && r[d] == 0.0;
    if (zero) continue;
    for (int d = 0; d < dim; ++d)
      if (r[d] != 0.0 && r[d] != 0.5 * out.box[d]) return false;  // not a half-box offset
    if (out.n_coset >= MAX_COSET) return false;
    double cc = 0;
    for (int d = 0; d < dim; ++d) {
      out.cw[out.n_coset][d] = r[d] != 0.0 ? out.box[d] : 0.0;
      cc += r[d] != 0.0 ? 0.25 * out.box[d] * out.box[d] : 0.0;
    }
    out.cc[out.n_coset++] = cc;
  }
  return true;
}

// Minimum over f in the box [c - 1/2, c + 1/2]^dim of f^T M f, M = A A^T the
// Gram matrix: the squared distance from the origin to the cell-shaped
// parallelepiped centred on the lattice point c.  Exact: the minimiser of a
// convex quadratic over a box has each coordinate either at a bound or
// stationary, so every free/lower/upper pattern is solved and the feasible
// ones compared.
double box_min_dist2(const double* M, int dim, const int* c) {
  double best = INFINITY;
  int patterns = 1;
  for (int d = 0; d < dim; ++d) patterns *= 3;
  for (int pat = 0; pat < patterns; ++pat) {
    int code[3] = {0, 0, 0};
    int t = pat;
    for (int d = 0; d < dim; ++d) {
      code[d] = t % 3;  // 0 free, 1 lower bound, 2 upper bound
      t /= 3;
    }
    double x[3] = {0, 0, 0};
    int fr[3], nf = 0;
    for (int d = 0; d < dim; ++d) {
      if (code[d] == 1) x[d] = c[d] - 0.5;
      else if (code[d] == 2) x[d] = c[d] + 0.5;
      else fr[nf++] = d;
    }
    if (nf > 0) {
      // solve M_FF x_F = -M_FX x_X by Gaussian elimination
      double m[3][4];
      for (int i = 0; i < nf; ++i) {
        double rhs = 0;
        for (int d = 0; d < dim; ++d)
          if (code[d] != 0) rhs -= M[fr[i] * 3 + d] * x[d];
        for (int j = 0; j < nf; ++j) m[i][j] = M[fr[i] * 3 + fr[j]];
        m[i][nf] = rhs;
      }
      bool ok = true;
      for (int i = 0; i < nf && ok; ++i) {
        int piv = i;
        for (int r = i + 1; r < nf; ++r)
          if (std::fabs(m[r][i]) > std::fabs(m[piv][i])) piv = r;
        if (std::fabs(m[piv][i]) < 1e-300) { ok = false; break; }
        for (int j = 0; j <= nf; ++j) std::swap(m[i][j], m[piv][j]);
        for (int r = 0; r < nf; ++r) {
          if (r == i) continue;
          double f = m[r][i] / m[i][i];
          for (int j = i; j <= nf; ++j) m[r][j] -= f * m[i][j];
        }
      }
      if (!ok) continue;
      bool feasible = true;
      for (int i = 0; i < nf; ++i) {
        double v = m[i][nf] / m[i][i];
        if (v < c[fr[i]] - 0.5 - 1e-12 || v > c[fr[i]] + 0.5 + 1e-12) feasible = false;
        x[fr[i]] = v;
      }
      if (!feasible) continue;
    }
    double q = 0;
    for (int i = 0; i < dim; ++i)
      for (int j = 0; j < dim; ++j) q += x[i] * M[i * 3 + j] * x[j];
    best = std::min(best, q);
  }
  return best;
}

// g(y) = erf(sqrt(y))/sqrt(y), an entire function of y with g(0) = 2/sqrt(pi).
double g_erf(double y) {
  if (y < 1e-300) return 2.0 / std::sqrt(kPi);
  const double r = std::sqrt(y);
  return std::erf(r) / r;
}

// Degree-deg polynomial in t = 2y/Y - 1 interpolating g at Chebyshev nodes of
// [0, Y], returned as monomial coefficients in t (Horner-ready).  The
// Chebyshev-to-monomial conversion runs in long double.
std::vector<double> fit_g(double Y, int deg) {
  const int n = deg + 1;
  std::vector<long double> c(n, 0.0L);
  for (int j = 0; j < n; ++j) {
    long double acc = 0.0L;
    for (int k = 0; k < n; ++k) {
      const long double th = kPi * (k + 0.5L) / n;
      acc += (long double)g_erf(0.5 * Y * (1.0 + double(std::cos(th)))) * std::cos(j * th);
    }
    c[j] = 2.0L * acc / n;
  }
  c[0] *= 0.5L;
  // T_0 = 1, T_1 = t, T_{j+1} = 2 t T_j - T_{j-1}
  std::vector<long double> tm1(n, 0.0L), t0(n, 0.0L), mono(n, 0.0L);
  tm1[0] = 1.0L;
  if (n > 1) t0[1] = 1.0L;
  mono[0] += c[0];
  if (n > 1) mono[1] += c[1];
  for (int j = 2; j < n; ++j) {
    std::vector<long double> tn(n, 0.0L);
    for (int i = 0; i < n; ++i) {
      if (i > 0) tn[i] += 2.0L * t0[i - 1];
      tn[i] -= tm1[i];
    }
    for (int i = 0; i < n; ++i) mono[i] += c[j] * tn[i];
    tm1 = t0;
    t0 = tn;
  }
  return std::vector<double>(mono.begin(), mono.end());
}

// Largest relative error of the Horner evaluation (in T) over [0, Y].
template <typename T>
double fit_error(const std::vector<double>& m, double Y) {
  double worst = 0.0;
  for (int k = 0; k <= 4000; ++k) {
    const double y = Y * k / 4000.0;
    const T t = T(2.0 * y / Y - 1.0);
    T p = T(m.back());
    for (int i = int(m.size()) - 2; i >= 0; --i) p = p * t + T(m[i]);
    const double ref = g_erf(y);
    worst = std::max(worst, std::fabs(double(p) - ref) / ref);
  }
  return worst;
}

}  // namespace

// ---------------------------------------------------------------------------

struct ewald_sys {
  int dim = 3;
  int n_mobile = 0, n_fixed = 0;
  int n_g = 0, n_seg = 0, n_shells = 0;
  int precision = 0, refresh_every = 0;
  bool has_jastrow = false;
  double r_ins = 0, e_const = 0;
  DevSys dev{};                      // scalars; device pointers once uploaded
  std::vector<uint32_t> seg_n;       // [n_seg]
  std::vector<int32_t> slot_n;       // slot-planar [n_slots][3]
  std::vector<double> w, ja;         // slot-planar [n_slots]
  std::vector<int32_t> shell;        // slot-planar, -1 for padding
  std::vector<double> shell_g2;      // |G|^2 of each shell
  std::vector<double> rho_fix;       // slot-planar [n_slots][2]
  std::vector<double> fixed_s, fixed_q, mobile_q;
  std::vector<int32_t> spin;         // [n_mobile] spin labels (u term)
  std::vector<double> wx, rho_fix1;  // layered: cross-plane weights, second plane's ions (slot-planar)
  std::vector<int32_t> fixed_layer;  // layered: plane of each ion
  std::vector<double> cand_cart;     // [n_cand][3] candidate offsets, caller's frame
  int device = -1;
  void* d_block = nullptr;
  DevSys dev_uploaded{};
  std::mutex mu;

  int n_slots() const { return n_seg * SEG; }
  ~ewald_sys() {
    if (d_block) dev_free(d_block);
  }
};

struct ewald_batch {
  std::vector<ewald_sys*> sys;
  std::vector<int> walker_sys;
  std::vector<DevWalker> walkers;
  std::vector<size_t> pos_offsets;
  size_t state_bytes = 0;
  void* d_sys = nullptr;
  void* d_walk = nullptr;
  LaunchBatch lb{};
  std::mutex mu;
  std::map<const void*, int> phase;  // state buffer -> 1 ready, 2 move pending
  ~ewald_batch() {
    if (d_sys) dev_free(d_sys);
    if (d_walk) dev_free(d_walk);
  }
};

// ---------------------------------------------------------------------------
// Per-call timers: invocations, host time and GPU time per ABI call, reported
// on request (the role of the paper's subroutine timers, Sec. 3.2).  GPU
// times come from event pairs resolved lazily (at a report, or when many are
// pending), so timing adds no synchronisation to the calls themselves.
namespace {

struct TimingRec {
  long calls = 0, gpu_calls = 0;
  double host_ms = 0.0, gpu_ms = 0.0;
};

struct TimingState {
  std::mutex mu;
  int on = -1;  // -1: EWALD_TIMING not read yet
  std::map<std::string, TimingRec> recs;
  std::vector<std::pair<std::string, void*>> pending;  // recorded event pairs
  std::vector<void*> pool;                             // free event pairs
};

TimingState& timing_state() {
  static TimingState* t = new TimingState;  // never destroyed: calls may come during exit
  return *t;
}

bool timing_on(TimingState& t) {
  if (t.on < 0) {
    const char* e = std::getenv("EWALD_TIMING");
    t.on = (e && *e && std::strcmp(e, "0") != 0) ? 1 : 0;
  }
  return t.on == 1;
}

void timing_resolve(TimingState& t) {
  for (auto& p : t.pending) {
    float ms = 0.f;
    if (event_pair_elapsed(p.second, &ms) == 0) {
      TimingRec& r = t.recs[p.first];
      r.gpu_ms += ms;
      r.gpu_calls += 1;
    }
    t.pool.push_back(p.second);
  }
  t.pending.clear();
}

double host_now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

namespace ewald {

// Timing never fails a call: an allocation failure here only loses the
// record (the guard's constructor and destructor catch everything).
CallTimer::CallTimer(const char* name, void* stream) noexcept : name_(name), stream_(stream) {
  try {
    TimingState& t = timing_state();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!timing_on(t)) return;
    on_ = true;
    t0_ = host_now_ms();
    int capturing = 0;
    if (stream_capturing(stream, &capturing) != 0 || capturing) return;  // no events inside a graph capture
    if (t.pool.empty()) {
      void* p = nullptr;
      if (event_pair_create(&p) == 0) {
        try {
          t.pool.push_back(p);
        } catch (...) {
          event_pair_destroy(p);
          throw;
        }
      }
    }
    if (t.pool.empty()) return;
    pair_ = t.pool.back();
    t.pool.pop_back();
    if (event_pair_record(pair_, 0, stream) != 0) {
      t.pool.push_back(pair_);  // capacity is there: the pair was just taken out
      pair_ = nullptr;
    }
  } catch (...) {
    // no record for this call's GPU time; a taken event pair is not leaked
    // (only the push into an empty pool can throw, before any pair is taken)
  }
}

CallTimer::~CallTimer() {
  if (!on_) return;
  try {
    const double host = host_now_ms() - t0_;
    TimingState& t = timing_state();
    std::lock_guard<std::mutex> lk(t.mu);
    if (pair_) {
      if (event_pair_record(pair_, 1, stream_) == 0) {
        t.pending.emplace_back(name_, pair_);
      } else {
        t.pool.push_back(pair_);
      }
      pair_ = nullptr;
    }
    TimingRec& r = t.recs[name_];
    r.calls += 1;
    r.host_ms += host;
    if (t.pending.size() >= 4096) timing_resolve(t);
  } catch (...) {
    if (pair_) event_pair_destroy(pair_);  // not recorded anywhere
  }
}

}  // namespace ewald

extern "C" {

const char* ewald_last_error(void) { return g_last_error.c_str(); }

ewald_status ewald_timing_enable(int on) {
  TimingState& t = timing_state();
  std::lock_guard<std::mutex> lk(t.mu);
  t.on = on ? 1 : 0;
  return EWALD_OK;
}

ewald_status ewald_timing_report(char* buf, size_t len, int reset) {
  if (!buf && len > 0) return fail(EWALD_E_ARG, "buf is NULL");
  TimingState& t = timing_state();
  std::lock_guard<std::mutex> lk(t.mu);
  timing_resolve(t);
  std::string out = "call calls gpu_calls gpu_ms_total gpu_ms_mean host_ms_total\n";
  for (const auto& kv : t.recs) {
    const TimingRec& r = kv.second;
    char line[256];
    std::snprintf(line, sizeof line, "%s %ld %ld %.6f %.6f %.6f\n", kv.first.c_str(), r.calls, r.gpu_calls,
                  r.gpu_ms, r.gpu_calls ? r.gpu_ms / double(r.gpu_calls) : 0.0, r.host_ms);
    out += line;
  }
  if (reset) t.recs.clear();
  if (len > 0) {
    const size_t n = std::min(out.size(), len - 1);
    std::memcpy(buf, out.data(), n);
    buf[n] = '\0';
    if (out.size() >= len) return fail(EWALD_E_ARG, "buf too small for the report (" + std::to_string(out.size() + 1) +
                                                     " bytes needed); truncated");
  }
  return EWALD_OK;
}

ewald_status ewald_setup(const ewald_sys_desc* desc, ewald_sys** out) try {
  if (!out) return fail(EWALD_E_ARG, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(EWALD_E_ARG, "desc is NULL");
  const int dim = desc->dim;
  if (dim != 2 && dim != 3) return fail(EWALD_E_ARG, "dim must be 2 or 3");
  if (desc->n_mobile < 1) return fail(EWALD_E_ARG, "n_mobile must be >= 1");
  if (desc->n_fixed < 0) return fail(EWALD_E_ARG, "n_fixed must be >= 0");
  if (desc->n_mobile + desc->n_fixed > EWALD_MAX_PARTICLES)
    return fail(EWALD_E_ARG, "n_mobile + n_fixed exceeds EWALD_MAX_PARTICLES");
  if (!desc->mobile_q) return fail(EWALD_E_ARG, "mobile_q is NULL");
  if (desc->n_fixed > 0 && (!desc->fixed_pos || !desc->fixed_q))
    return fail(EWALD_E_ARG, "fixed_pos/fixed_q NULL with n_fixed > 0");
  if (desc->precision != EWALD_FP64 && desc->precision != EWALD_FP32_MIXED)
    return fail(EWALD_E_ARG, "unknown precision");
  if (desc->refresh_every < 0) return fail(EWALD_E_ARG, "refresh_every must be >= 0");
  if (desc->n_jastrow < 0) return fail(EWALD_E_ARG, "n_jastrow must be >= 0");
  if (desc->n_jastrow > 0 && !desc->jastrow_a) return fail(EWALD_E_ARG, "jastrow_a is NULL");
  for (int i = 0; i < desc->n_mobile; ++i)
    if (!is_fin(desc->mobile_q[i])) return fail(EWALD_E_ARG, "non-finite mobile charge");
  for (int i = 0; i < desc->n_fixed; ++i) {
    if (!is_fin(desc->fixed_q[i])) return fail(EWALD_E_ARG, "non-finite fixed charge");
    for (int d = 0; d < dim; ++d)
      if (!is_fin(desc->fixed_pos[i * dim + d])) return fail(EWALD_E_ARG, "non-finite fixed position");
  }
  for (int i = 0; i < desc->n_jastrow; ++i)
    if (!is_fin(desc->jastrow_a[i])) return fail(EWALD_E_ARG, "non-finite Jastrow coefficient");
  const int u_terms = desc->u_terms;
  if (u_terms < 0) return fail(EWALD_E_ARG, "u_terms must be >= 0");
  if (u_terms > 0) {
    if (!desc->u_alpha) return fail(EWALD_E_ARG, "u_alpha is NULL");
    if (desc->u_C < 1) return fail(EWALD_E_ARG, "u_C must be >= 1");
    if (u_terms - 1 + desc->u_C > UDEG) return fail(EWALD_E_ARG, "u_terms - 1 + u_C exceeds 15");
    for (int i = 0; i < 2 * u_terms; ++i)
      if (!is_fin(desc->u_alpha[i])) return fail(EWALD_E_ARG, "non-finite u coefficient");
    if (desc->mobile_spin)
      for (int i = 0; i < desc->n_mobile; ++i)
        if (desc->mobile_spin[i] != 0 && desc->mobile_spin[i] != 1)
          return fail(EWALD_E_ARG, "spin labels must be 0 or 1");
  }

  // ---- lattice ----
  double A[9] = {0};
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) {
      A[i * 3 + j] = desc->lattice[i][j];
      if (!is_fin(A[i * 3 + j])) return fail(EWALD_E_LATTICE, "non-finite lattice");
    }
  double norms[3] = {0, 0, 0};
  double prod = 1;
  for (int i = 0; i < dim; ++i) {
    for (int j = 0; j < dim; ++j) norms[i] += A[i * 3 + j] * A[i * 3 + j];
    norms[i] = std::sqrt(norms[i]);
    prod *= norms[i];
  }
  const double det = det_n(A, dim);
  if (!(prod > 0) || std::fabs(det) <= 1e-10 * prod) return fail(EWALD_E_LATTICE, "singular lattice");
  const double measure = std::fabs(det);  // volume (3D) or area (2D)
  double Ainv[9];
  inverse_n(A, dim, Ainv);
  // reciprocal vectors b_i = 2 pi (A^-T)_i: B[i][e] = 2 pi Ainv[e][i]
  double Bm[9] = {0};
  double bnorm[3] = {0, 0, 0};
  for (int i = 0; i < dim; ++i) {
    for (int e = 0; e < dim; ++e) {
      Bm[i * 3 + e] = 2 * kPi * Ainv[e * 3 + i];
      bnorm[i] += Bm[i * 3 + e] * Bm[i * 3 + e];
    }
    bnorm[i] = std::sqrt(bnorm[i]);
  }
  double M[9] = {0};  // Gram matrix A A^T
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j)
      for (int e = 0; e < dim; ++e) M[i * 3 + j] += A[i * 3 + e] * A[j * 3 + e];

  // inscribed radius: half the shortest nonzero lattice vector.  A vector of
  // length <= l has |n_i| <= l |b_i| / 2 pi.
  double shortest = *std::min_element(norms, norms + dim);
  int bound[3] = {0, 0, 0};
  for (int i = 0; i < dim; ++i) bound[i] = int(std::floor(shortest * bnorm[i] / (2 * kPi))) + 1;
  for (int i = -bound[0]; i <= bound[0]; ++i)
    for (int j = -bound[1]; j <= bound[1]; ++j)
      for (int k = -(dim == 3 ? bound[2] : 0); k <= (dim == 3 ? bound[2] : 0); ++k) {
        if (i == 0 && j == 0 && k == 0) continue;
        double v2 = 0;
        for (int e = 0; e < dim; ++e) {
          double v = i * A[e] + j * A[3 + e] + k * A[6 + e];
          v2 += v * v;
        }
        shortest = std::min(shortest, std::sqrt(v2));
      }
  const double r_ins = 0.5 * shortest;

  const double alpha = desc->alpha, r_cut = desc->r_cut, g_cut = desc->g_cut;
  if (!is_fin(alpha) || !(alpha > 0)) return fail(EWALD_E_ARG, "alpha must be > 0");
  if (!is_fin(r_cut) || !(r_cut > 0)) return fail(EWALD_E_RCUT, "r_cut must be > 0");
  if (r_cut > r_ins) return fail(EWALD_E_RCUT, "r_cut exceeds the inscribed radius (half the shortest lattice vector)");
  if (!is_fin(g_cut) || !(g_cut > 0)) return fail(EWALD_E_GCUT, "g_cut must be > 0");
  const int n_layers = desc->n_layers;
  if (n_layers < 0 || n_layers > 2) return fail(EWALD_E_ARG, "n_layers must be 0, 1 or 2");
  const bool layered = n_layers == 2;
  if (layered) {
    if (dim != 2) return fail(EWALD_E_ARG, "layers need a two-dimensional cell");
    if (desc->n_jastrow > 0 || u_terms > 0) return fail(EWALD_E_ARG, "layered systems take no Jastrow terms");
    if (desc->n_mobile_layer0 < 0 || desc->n_mobile_layer0 > desc->n_mobile)
      return fail(EWALD_E_ARG, "n_mobile_layer0 must be in [0, n_mobile]");
    if (!is_fin(desc->layer_z[0]) || !is_fin(desc->layer_z[1])) return fail(EWALD_E_ARG, "non-finite layer height");
    if (desc->fixed_layer)
      for (int i = 0; i < desc->n_fixed; ++i)
        if (desc->fixed_layer[i] != 0 && desc->fixed_layer[i] != 1)
          return fail(EWALD_E_ARG, "fixed_layer entries must be 0 or 1");
  }
  const double u_cut = u_terms > 0 ? desc->u_cutoff : 0.0;
  if (u_terms > 0 && (!is_fin(u_cut) || !(u_cut > 0) || u_cut > r_ins * (1.0 + 1e-12)))
    return fail(EWALD_E_RCUT, "u_cutoff must be in (0, r_inscribed]");
  // minimum images are resolved exactly up to this distance
  const double r_img = std::max(r_cut, u_cut);
  // the pair potential's erf part is one polynomial on [0, r_cut]; it is
  // built for alpha r_cut <= 5.5, where erfc(alpha r_cut) < 1e-14 already
  if (alpha * r_cut > 5.5)
    return fail(EWALD_E_RCUT, "alpha * r_cut above 5.5 (the real-space sum is converged below 1e-14 there)");

  // ---- G set: nonzero n with |n B| <= g_cut; the ball spans |n_d| <= g_cut |a_d| / 2 pi ----
  int nb[3] = {0, 0, 0};
  for (int d = 0; d < dim; ++d) {
    double ext = g_cut * norms[d] / (2 * kPi);
    if (ext > EWALD_MAX_NRED) return fail(EWALD_E_GCUT, "g_cut too large for the reduced-index range");
    nb[d] = int(std::ceil(ext));
  }
  const double lim = g_cut * g_cut * (1.0 + 1e-12);
  struct GV { int n[3]; double g2; };
  std::vector<GV> half;
  for (int i = -nb[0]; i <= nb[0]; ++i)
    for (int j = -nb[1]; j <= nb[1]; ++j)
      for (int k = -(dim == 3 ? nb[2] : 0); k <= (dim == 3 ? nb[2] : 0); ++k) {
        int n[3] = {i, j, k};
        // half set: first nonzero reduced coordinate positive
        int first = 0;
        for (int d = 0; d < dim; ++d)
          if (n[d] != 0) { first = n[d]; break; }
        if (first <= 0) continue;
        double g2 = 0;
        for (int e = 0; e < dim; ++e) {
          double ge = 0;
          for (int d = 0; d < dim; ++d) ge += n[d] * Bm[d * 3 + e];
          g2 += ge * ge;
        }
        if (g2 <= lim) half.push_back({{i, j, k}, g2});
      }
  if (half.empty()) return fail(EWALD_E_GCUT, "no reciprocal lattice vector within g_cut");
  const int last = dim - 1;
  // columns: equal leading coordinates, runs along the last coordinate
  std::sort(half.begin(), half.end(), [&](const GV& a, const GV& b) {
    for (int d = 0; d < dim; ++d)
      if (a.n[d] != b.n[d]) return a.n[d] < b.n[d];
    return false;
  });
  struct Seg { int n[3]; };
  std::vector<Seg> segs;
  std::vector<std::vector<double>> seg_g2;  // g2 per slot (NaN: padding)
  for (size_t a = 0; a < half.size();) {
    size_t b = a;
    while (b < half.size()) {
      bool same = true;
      for (int d = 0; d < last; ++d) same = same && half[b].n[d] == half[a].n[d];
      if (!same) break;
      ++b;
    }
    // [a, b) is one column; its last coordinates are consecutive (a convex set
    // meets a line in an interval)
    for (size_t t = a + 1; t < b; ++t)
      if (half[t].n[last] != half[t - 1].n[last] + 1)
        return fail(EWALD_E_GCUT, "internal: non-contiguous G column");
    for (size_t t = a; t < b; t += SEG) {
      Seg s;
      std::copy(half[t].n, half[t].n + 3, s.n);
      segs.push_back(s);
      std::vector<double> g2(SEG, std::nan(""));
      for (int j = 0; j < SEG && t + j < b; ++j) g2[j] = half[t + j].g2;
      seg_g2.push_back(g2);
    }
    a = b;
  }
  const int n_seg = int(segs.size());
  if (n_seg > EWALD_MAX_SEGMENTS) return fail(EWALD_E_GCUT, "G set exceeds EWALD_MAX_SEGMENTS");
  const int n_slots = n_seg * SEG;

  // shells of equal |G|^2 (relative tolerance 1e-9), ascending
  std::vector<double> g2s;
  for (auto& g : half) g2s.push_back(g.g2);
  std::sort(g2s.begin(), g2s.end());
  std::vector<double> shells;
  for (double v : g2s)
    if (shells.empty() || v > shells.back() * (1.0 + 1e-9)) shells.push_back(v);

  std::unique_ptr<ewald_sys> S(new ewald_sys());
  S->dim = dim;
  S->n_mobile = desc->n_mobile;
  S->n_fixed = desc->n_fixed;
  S->n_g = int(half.size());
  S->n_seg = n_seg;
  S->n_shells = int(shells.size());
  S->precision = desc->precision;
  S->refresh_every = desc->refresh_every;
  S->has_jastrow = desc->n_jastrow > 0 || u_terms > 0;
  S->r_ins = r_ins;
  S->seg_n.resize(n_seg);
  S->slot_n.assign(size_t(n_slots) * 3, 0);
  S->w.assign(n_slots, 0.0);
  S->ja.assign(n_slots, 0.0);
  S->shell.assign(n_slots, -1);
  S->rho_fix.assign(size_t(n_slots) * 2, 0.0);
  if (layered) {
    S->wx.assign(n_slots, 0.0);
    S->rho_fix1.assign(size_t(n_slots) * 2, 0.0);
    S->fixed_layer.assign(size_t(desc->n_fixed), 0);
    if (desc->fixed_layer) std::copy(desc->fixed_layer, desc->fixed_layer + desc->n_fixed, S->fixed_layer.begin());
  }
  int nmax[3] = {0, 0, 0};
  for (auto& g : half)
    for (int d = 0; d < dim; ++d) nmax[d] = std::max(nmax[d], std::abs(g.n[d]));
  double jlap_c = 0.0;  // sum over the half set of a_s(G) |G|^2
  for (int s = 0; s < n_seg; ++s) {
    const Seg& sg = segs[s];
    S->seg_n[s] = pack_n(sg.n[0], sg.n[1], sg.n[2]);
    for (int j = 0; j < SEG; ++j) {
      const size_t slot = size_t(j) * n_seg + s;
      int n[3] = {sg.n[0], sg.n[1], sg.n[2]};
      n[last] += j;
      for (int d = 0; d < 3; ++d) S->slot_n[slot * 3 + d] = n[d];
      const double g2 = seg_g2[s][j];
      if (std::isnan(g2)) continue;  // padding slot: weight 0
      const double g = std::sqrt(g2);
      S->w[slot] = (dim == 3) ? 4 * kPi / measure * std::exp(-g2 / (4 * alpha * alpha)) / g2
                              : 2 * kPi / measure * std::erfc(g / (2 * alpha)) / g;
      if (layered) {  // (pi/A) [e^{dG} erfc(G/2a + da) + e^{-dG} erfc(G/2a - da)] / G, in long double
        const long double d = std::fabs((long double)desc->layer_z[1] - (long double)desc->layer_z[0]);
        const long double gl = g, al = alpha;
        const long double f = std::exp(d * gl) * std::erfc(gl / (2 * al) + d * al) +
                              std::exp(-d * gl) * std::erfc(gl / (2 * al) - d * al);
        S->wx[slot] = double((long double)kPi / measure * f / gl);
      }
      int sh = int(std::lower_bound(shells.begin(), shells.end(), g2 * (1.0 - 1e-9)) - shells.begin());
      S->shell[slot] = sh;
      S->ja[slot] = (sh < desc->n_jastrow) ? desc->jastrow_a[sh] : 0.0;
      jlap_c += S->ja[slot] * g2;
    }
  }
  S->shell_g2 = shells;

  // ---- charges, fixed ions ----
  S->mobile_q.assign(desc->mobile_q, desc->mobile_q + desc->n_mobile);
  S->fixed_q.assign(desc->fixed_q, desc->fixed_q + desc->n_fixed);
  S->fixed_s.assign(size_t(desc->n_fixed) * dim, 0.0);
  for (int I = 0; I < desc->n_fixed; ++I)
    for (int d = 0; d < dim; ++d) {
      double v = 0;
      for (int e = 0; e < dim; ++e) v += desc->fixed_pos[I * dim + e] * Ainv[e * 3 + d];
      S->fixed_s[I * dim + d] = wrap01(v);
    }
  for (int I = 0; I < desc->n_fixed; ++I) {
    for (int slot = 0; slot < n_slots; ++slot) {
      double x = 0;
      for (int d = 0; d < dim; ++d) x += S->slot_n[slot * 3 + d] * S->fixed_s[I * dim + d];
      x -= std::nearbyint(x);
      std::vector<double>& rf = (layered && S->fixed_layer[I] == 1) ? S->rho_fix1 : S->rho_fix;
      rf[2 * slot] += S->fixed_q[I] * std::cos(2 * kPi * x);
      rf[2 * slot + 1] += S->fixed_q[I] * std::sin(2 * kPi * x);
    }
  }

  // ---- minimum-image candidates: lattice points c != 0 whose cell-shaped box
  // comes within r_img = max(r_cut, L_u) of the origin (one of each +-pair) ----
  std::vector<double> cand;
  const int cr = 3;
  for (int i = -cr; i <= cr; ++i)
    for (int j = -cr; j <= cr; ++j)
      for (int k = -(dim == 3 ? cr : 0); k <= (dim == 3 ? cr : 0); ++k) {
        int c[3] = {i, j, k};
        int first = 0;
        for (int d = 0; d < dim; ++d)
          if (c[d] != 0) { first = c[d]; break; }
        if (first <= 0) continue;
        // a box that only touches the cutoff sphere holds no point strictly
        // inside it (the real-space test is |r| < r_cut)
        double d2 = box_min_dist2(M, dim, c);
        if (d2 < r_img * r_img * (1.0 - 1e-12)) {
          bool edge = false;
          for (int d = 0; d < dim; ++d) edge = edge || std::abs(c[d]) == cr;
          if (edge) return fail(EWALD_E_RCUT, "internal: candidate search range too small");
          double v[3] = {0, 0, 0}, v2 = 0;
          for (int e = 0; e < dim; ++e) {
            for (int d = 0; d < dim; ++d) v[e] += c[d] * A[d * 3 + e];
            v2 += v[e] * v[e];
          }
          cand.insert(cand.end(), {v[0], v[1], v[2], v2});
        }
      }
  const int n_cand = int(cand.size() / 4);
  if (n_cand > MAX_CAND) return fail(EWALD_E_RCUT, "too many minimum-image candidates for this cell");

  // ---- constants ----
  double q2 = 0, qt = 0;
  for (double q : S->mobile_q) { q2 += q * q; qt += q; }
  for (double q : S->fixed_q) { q2 += q * q; qt += q; }
  const double e_self = -alpha / std::sqrt(kPi) * q2;
  double e_bg = (dim == 3) ? -kPi / (2 * measure * alpha * alpha) * qt * qt
                           : -std::sqrt(kPi) / (measure * alpha) * qt * qt;
  const double dz = layered ? desc->layer_z[1] - desc->layer_z[0] : 0.0;
  if (layered) {  // 1/2 sum_{l,m} Q_l Q_m c(z_l - z_m)
    double Q[2] = {0, 0};
    for (int i = 0; i < desc->n_mobile; ++i) Q[i >= desc->n_mobile_layer0 ? 1 : 0] += S->mobile_q[i];
    for (int I = 0; I < desc->n_fixed; ++I) Q[S->fixed_layer[I]] += S->fixed_q[I];
    auto c = [&](double z) {
      return -2 * kPi / measure * (z * std::erf(z * alpha) + std::exp(-alpha * alpha * z * z) / (alpha * std::sqrt(kPi)));
    };
    e_bg = 0.5 * (Q[0] * Q[0] + Q[1] * Q[1]) * c(0.0) + Q[0] * Q[1] * c(dz);
  }
  // ion-ion real-space pairs (the ions never move); images by brute force
  double e_ii = 0;
  for (int I = 0; I < desc->n_fixed; ++I)
    for (int J = I + 1; J < desc->n_fixed; ++J) {
      double f[3] = {0, 0, 0};
      for (int d = 0; d < dim; ++d) {
        f[d] = S->fixed_s[I * dim + d] - S->fixed_s[J * dim + d];
        f[d] -= std::nearbyint(f[d]);
      }
      double best = INFINITY;
      for (int i = -2; i <= 2; ++i)
        for (int j = -2; j <= 2; ++j)
          for (int k = -(dim == 3 ? 2 : 0); k <= (dim == 3 ? 2 : 0); ++k) {
            int c[3] = {i, j, k};
            double r2 = 0;
            for (int e = 0; e < dim; ++e) {
              double v = 0;
              for (int d = 0; d < dim; ++d) v += (f[d] + c[d]) * A[d * 3 + e];
              r2 += v * v;
            }
            best = std::min(best, r2);
          }
      if (layered && S->fixed_layer[I] != S->fixed_layer[J]) best += dz * dz;
      if (best < r_cut * r_cut) {
        double r = std::sqrt(best);
        e_ii += S->fixed_q[I] * S->fixed_q[J] * std::erfc(alpha * r) / r;
      }
    }
  S->e_const = e_self + e_bg + e_ii;

  // polynomial for erf(alpha r)/(alpha r) on r in [0, r_cut]
  const double Y = alpha * alpha * r_cut * r_cut;
  const int deg64 = (Y <= 8.0) ? 16 : 32;
  const int deg32 = (Y <= 8.0) ? 12 : 22;
  const std::vector<double> p64 = fit_g(Y, deg64);
  const std::vector<double> p32 = fit_g(Y, deg32);
  if (fit_error<double>(p64, Y) > 1e-12 || fit_error<float>(p32, Y) > 1e-6)
    return fail(EWALD_E_RCUT, "internal: pair-potential polynomial inaccurate");
  // rows of the lattice in an orthonormal frame where they are lower-triangular
  // (Gram-Schmidt); distances are invariant under this rotation
  double Lrot[9] = {0};
  {
    double e[3][3] = {{0}};
    for (int i = 0; i < dim; ++i) {
      double v[3] = {A[i * 3], A[i * 3 + 1], A[i * 3 + 2]};
      for (int j = 0; j < i; ++j) {
        double d = v[0] * e[j][0] + v[1] * e[j][1] + v[2] * e[j][2];
        for (int x = 0; x < 3; ++x) v[x] -= d * e[j][x];
      }
      double nv = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      for (int x = 0; x < 3; ++x) e[i][x] = v[x] / nv;
    }
    for (int i = 0; i < dim; ++i)
      for (int j = 0; j <= i; ++j)
        Lrot[i * 3 + j] = A[i * 3] * e[j][0] + A[i * 3 + 1] * e[j][1] + A[i * 3 + 2] * e[j][2];
    for (int i = 0; i < 3; ++i)
      for (int x = 0; x < 3; ++x) S->dev.El[i * 3 + x] = e[i][x];
  }

  for (int c = 0; c < n_cand; ++c)
    for (int e = 0; e < 3; ++e) S->cand_cart.push_back(cand[c * 4 + e]);

  DevSys& D = S->dev;
  D.dim = dim;
  D.n_mobile = S->n_mobile;
  D.n_fixed = S->n_fixed;
  D.n_seg = n_seg;
  for (int d = 0; d < 3; ++d) D.nmax[d] = nmax[d];
  D.nm = std::max(nmax[0], std::max(nmax[1], nmax[2]));
  D.n_cand = n_cand;
  D.has_jastrow = S->has_jastrow ? 1 : 0;
  D.refresh_every = S->refresh_every;
  D.precision = S->precision;
  std::copy(A, A + 9, D.A);
  std::copy(Ainv, Ainv + 9, D.Ainv);
  std::copy(Lrot, Lrot + 9, D.Lrot);
  D.alpha = alpha;
  D.rc2 = r_cut * r_cut;
  D.poly_scale = 2.0 / (r_cut * r_cut);
  D.poly_deg = deg64;
  for (int i = 0; i <= POLY_MAX; ++i) D.p64[i] = i <= deg64 ? p64[i] : 0.0;
  for (int i = 0; i <= POLY32_MAX; ++i) D.p32[i] = i <= deg32 ? float(p32[i]) : 0.0f;
  D.e_const = S->e_const;
  for (int t = 0; t < 9; ++t) D.B[t] = Bm[t];
  D.jlap_c = jlap_c;
  // candidate offsets in the rotated frame: c . Lrot
  for (int c = 0; c < n_cand; ++c) {
    int ci[3] = {0, 0, 0};
    // recover the integer combination: cand = ci . A  =>  ci = cand . Ainv
    for (int d = 0; d < dim; ++d) {
      double v = 0;
      for (int e = 0; e < dim; ++e) v += cand[c * 4 + e] * Ainv[e * 3 + d];
      ci[d] = int(std::lround(v));
    }
    double v2 = 0;
    for (int e = 0; e < 3; ++e) {
      double v = 0;
      for (int d = 0; d < dim; ++d) v += ci[d] * Lrot[d * 3 + e];
      D.cand[c][e] = v;
      v2 += v * v;
    }
    D.cand[c][3] = v2;
  }
  // Jastrow u term: sum_l alpha_l r^l (r - L)^C = L^C sum_l alpha_l L^l t^l (t - 1)^C
  // in powers of t = r / L (long double), per channel; channel 1 stored as
  // its difference from channel 0
  D.n_layers = layered ? 2 : 1;
  D.n0 = layered ? desc->n_mobile_layer0 : S->n_mobile;
  D.dz2 = dz * dz;
  D.has_u = u_terms > 0 ? 1 : 0;
  if (u_terms > 0) {
    const int C = desc->u_C;
    long double beta[2][UDEG + 1] = {{0}};
    for (int c = 0; c < 2; ++c)
      for (int l = 0; l < u_terms; ++l) {
        long double binom = 1.0L;  // C choose k
        for (int k = 0; k <= C; ++k) {
          const long double sgn = ((C - k) & 1) ? -1.0L : 1.0L;
          beta[c][l + k] += (long double)desc->u_alpha[c * u_terms + l] * std::pow((long double)u_cut, l + C) *
                            binom * sgn;
          binom = binom * (C - k) / (k + 1);
        }
      }
    for (int m = 0; m <= UDEG; ++m) {
      D.u_c0[m] = double(beta[0][m]);
      D.u_dc[m] = double(beta[1][m] - beta[0][m]);
    }
    D.u_cut2 = u_cut * u_cut;
    D.u_icut = 1.0 / u_cut;
    S->spin.assign(size_t(desc->n_mobile), 0);
    if (desc->mobile_spin) std::copy(desc->mobile_spin, desc->mobile_spin + desc->n_mobile, S->spin.begin());
  }
  OrthoFrame of;
  D.ortho = ortho_frame(A, dim, of) ? 1 : 0;
  if (D.ortho) {
    std::copy(of.F, of.F + 9, D.F);
    std::copy(of.E, of.E + 9, D.Eo);
    for (int d = 0; d < 3; ++d) {
      D.box[d] = of.box[d];
      D.ibox[d] = of.box[d] > 0 ? 1.0 / of.box[d] : 0.0;
    }
    D.n_coset = of.n_coset;
    for (int c = 0; c < MAX_COSET; ++c) {
      for (int d = 0; d < 3; ++d) D.cw[c][d] = of.cw[c][d];
      // an absent coset never gives the nearest image
      D.cc[c] = c < of.n_coset ? of.cc[c] : HUGE_VAL;
    }
  }
  *out = S.release();
  return EWALD_OK;
} catch (const std::bad_alloc&) {
  return fail(EWALD_E_NOMEM, "host allocation failed");
} catch (...) {
  return fail(EWALD_E_ARG, "unexpected error in ewald_setup");
}

ewald_status ewald_sys_query(const ewald_sys* s, int* n_g, int* n_slots, int* n_shells,
                             double* r_inscribed, double* e_const) {
  if (!s) return fail(EWALD_E_ARG, "sys is NULL");
  if (n_g) *n_g = s->n_g;
  if (n_slots) *n_slots = s->n_slots();
  if (n_shells) *n_shells = s->n_shells;
  if (r_inscribed) *r_inscribed = s->r_ins;
  if (e_const) *e_const = s->e_const;
  return EWALD_OK;
}

ewald_status ewald_sys_tables(const ewald_sys* s, int32_t* n, double* weight, double* jastrow,
                              int32_t* shell) {
  if (!s) return fail(EWALD_E_ARG, "sys is NULL");
  const size_t ns = size_t(s->n_slots());
  if (n) std::memcpy(n, s->slot_n.data(), ns * 3 * sizeof(int32_t));
  if (weight) std::memcpy(weight, s->w.data(), ns * sizeof(double));
  if (jastrow) std::memcpy(jastrow, s->ja.data(), ns * sizeof(double));
  if (shell) std::memcpy(shell, s->shell.data(), ns * sizeof(int32_t));
  return EWALD_OK;
}

ewald_status ewald_sys_candidates(const ewald_sys* s, int* n_cand, double* cand) {
  if (!s) return fail(EWALD_E_ARG, "sys is NULL");
  if (n_cand) *n_cand = s->dev.n_cand;
  if (cand)
    for (int c = 0; c < s->dev.n_cand; ++c)
      for (int e = 0; e < 3; ++e) cand[c * 3 + e] = s->cand_cart[c * 3 + e];
  return EWALD_OK;
}

ewald_status ewald_sys_geometry(const ewald_sys* s, int* index, double* box) {
  if (!s) return fail(EWALD_E_ARG, "sys is NULL");
  if (index) *index = s->dev.ortho ? s->dev.n_coset + 1 : 0;
  if (box)
    for (int d = 0; d < 3; ++d) box[d] = s->dev.ortho ? s->dev.box[d] : 0.0;
  return EWALD_OK;
}

void ewald_sys_destroy(ewald_sys* s) { delete s; }

}  // extern "C"

namespace {

// Copy one system's tables to the current device (once).
ewald_status upload_sys(ewald_sys* s, int device) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->d_block) {
    if (s->device != device) return fail(EWALD_E_ARG, "system already uploaded to another device");
    return EWALD_OK;
  }
  const size_t ns = size_t(s->n_slots());
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t o_seg = take(s->seg_n.size() * 4);
  const size_t o_w = take(ns * 8);
  const size_t o_ja = take(ns * 8);
  const size_t o_rf = take(ns * 16);
  const size_t o_fs = take(std::max<size_t>(1, s->fixed_s.size()) * 8);
  const size_t o_fq = take(std::max<size_t>(1, s->fixed_q.size()) * 8);
  const size_t o_mq = take(s->mobile_q.size() * 8);
  const size_t o_sp = take(std::max<size_t>(1, s->spin.size()) * 4);
  const size_t o_wx = take(s->wx.size() * 8);
  const size_t o_rf1 = take(s->rho_fix1.size() * 8);
  const size_t o_fl = take(std::max<size_t>(1, s->fixed_layer.size()) * 4);
  // shell table: (w, a) per shell and a zero entry for padding slots
  const int n_wtab = s->n_shells + 1;
  std::vector<double> wa(size_t(n_wtab) * 2, 0.0);
  std::vector<uint16_t> sl(ns, uint16_t(n_wtab - 1));
  const bool sh16 = n_wtab <= 65535;
  for (size_t g = 0; g < ns; ++g) {
    const int sh = s->shell[g];
    if (sh < 0) continue;
    wa[2 * size_t(sh)] = s->w[g];
    wa[2 * size_t(sh) + 1] = s->ja[g];
    if (sh16) sl[g] = uint16_t(sh);
  }
  // a_s |G_s|^2 per shell for the Jastrow Laplacian
  std::vector<double> jg2(size_t(n_wtab), 0.0);
  for (size_t g = 0; g < ns; ++g) {
    const int sh = s->shell[g];
    if (sh >= 0) jg2[size_t(sh)] = s->ja[g] * s->shell_g2[size_t(sh)];
  }
  // cross-plane weight per shell (layered systems)
  std::vector<double> wxt;
  if (!s->wx.empty()) {
    wxt.assign(size_t(n_wtab), 0.0);
    for (size_t g = 0; g < ns; ++g)
      if (s->shell[g] >= 0) wxt[size_t(s->shell[g])] = s->wx[g];
  }
  const size_t o_wxt = take(std::max<size_t>(1, wxt.size()) * 8);
  const size_t o_wa = take(wa.size() * 8);
  const size_t o_jg = take(jg2.size() * 8);
  const size_t o_sl = take(sl.size() * 2);
  std::vector<char> host(off, 0);
  std::memcpy(host.data() + o_seg, s->seg_n.data(), s->seg_n.size() * 4);
  std::memcpy(host.data() + o_w, s->w.data(), ns * 8);
  std::memcpy(host.data() + o_ja, s->ja.data(), ns * 8);
  std::memcpy(host.data() + o_rf, s->rho_fix.data(), ns * 16);
  if (!s->fixed_s.empty()) std::memcpy(host.data() + o_fs, s->fixed_s.data(), s->fixed_s.size() * 8);
  if (!s->fixed_q.empty()) std::memcpy(host.data() + o_fq, s->fixed_q.data(), s->fixed_q.size() * 8);
  std::memcpy(host.data() + o_mq, s->mobile_q.data(), s->mobile_q.size() * 8);
  if (!s->spin.empty()) std::memcpy(host.data() + o_sp, s->spin.data(), s->spin.size() * 4);
  if (!s->wx.empty()) std::memcpy(host.data() + o_wx, s->wx.data(), s->wx.size() * 8);
  if (!wxt.empty()) std::memcpy(host.data() + o_wxt, wxt.data(), wxt.size() * 8);
  if (!s->rho_fix1.empty()) std::memcpy(host.data() + o_rf1, s->rho_fix1.data(), s->rho_fix1.size() * 8);
  if (!s->fixed_layer.empty()) std::memcpy(host.data() + o_fl, s->fixed_layer.data(), s->fixed_layer.size() * 4);
  std::memcpy(host.data() + o_wa, wa.data(), wa.size() * 8);
  std::memcpy(host.data() + o_jg, jg2.data(), jg2.size() * 8);
  std::memcpy(host.data() + o_sl, sl.data(), sl.size() * 2);
  void* d = nullptr;
  int rc = dev_alloc(&d, off);
  if (rc) return fail(EWALD_E_NOMEM, std::string("device allocation failed: ") + dev_error_string(rc));
  rc = dev_upload(d, host.data(), off);
  if (rc) {
    dev_free(d);
    return fail(EWALD_E_HIP, std::string("table upload failed: ") + dev_error_string(rc));
  }
  char* base = static_cast<char*>(d);
  DevSys D = s->dev;
  D.seg_n = reinterpret_cast<const uint32_t*>(base + o_seg);
  D.w = reinterpret_cast<const double*>(base + o_w);
  D.ja = s->has_jastrow ? reinterpret_cast<const double*>(base + o_ja) : nullptr;
  D.rho_fix = reinterpret_cast<const double*>(base + o_rf);
  D.fixed_s = reinterpret_cast<const double*>(base + o_fs);
  D.fixed_q = reinterpret_cast<const double*>(base + o_fq);
  D.mobile_q = reinterpret_cast<const double*>(base + o_mq);
  D.spin = s->spin.empty() ? nullptr : reinterpret_cast<const int32_t*>(base + o_sp);
  D.wx = s->wx.empty() ? nullptr : reinterpret_cast<const double*>(base + o_wx);
  D.wx_tab = wxt.empty() ? nullptr : reinterpret_cast<const double*>(base + o_wxt);
  D.rho_fix1 = s->rho_fix1.empty() ? nullptr : reinterpret_cast<const double*>(base + o_rf1);
  D.fixed_layer = s->fixed_layer.empty() ? nullptr : reinterpret_cast<const int32_t*>(base + o_fl);
  D.wa_tab = reinterpret_cast<const double*>(base + o_wa);
  D.jg2_tab = reinterpret_cast<const double*>(base + o_jg);
  D.slot_shell = reinterpret_cast<const uint16_t*>(base + o_sl);
  D.n_wtab = n_wtab;
  D.wtab_lds = (sh16 && n_wtab <= WTAB_MAX) ? 1 : 0;
  s->dev_uploaded = D;
  s->d_block = d;
  s->device = device;
  return EWALD_OK;
}

ewald_status check_state(ewald_batch* b, const void* state, int need, int set) {
  std::lock_guard<std::mutex> lk(b->mu);
  auto it = b->phase.find(state);
  int ph = it == b->phase.end() ? 0 : it->second;
  if (need == 1 && ph < 1) return fail(EWALD_E_STATE, "state not initialised: call ewald_energy_batch first");
  if (need == 2 && ph != 2) return fail(EWALD_E_STATE, "no pending move: call ewald_move_delta_batch first");
  if (need == 3 && ph != 1)
    return fail(EWALD_E_STATE, ph == 0 ? "state not initialised: call ewald_energy_batch first"
                                       : "a move is pending: accept or reject it first");
  if (set >= 0) b->phase[state] = set;
  return EWALD_OK;
}

ewald_status launch_status(int rc, const char* what) {
  if (rc == 0) return EWALD_OK;
  return fail(EWALD_E_HIP, std::string(what) + " launch failed: " + dev_error_string(rc));
}

}  // namespace

extern "C" {

ewald_status ewald_batch_create(ewald_sys* const* sys, int n_sys, const int* walker_sys,
                                int n_walkers, ewald_batch** out) try {
  if (!out) return fail(EWALD_E_ARG, "out is NULL");
  *out = nullptr;
  if (!sys || n_sys < 1) return fail(EWALD_E_ARG, "need at least one system");
  if (!walker_sys || n_walkers < 1) return fail(EWALD_E_ARG, "need at least one walker");
  for (int i = 0; i < n_sys; ++i)
    if (!sys[i]) return fail(EWALD_E_ARG, "NULL system");
  for (int i = 1; i < n_sys; ++i) {
    if (sys[i]->dim != sys[0]->dim) return fail(EWALD_E_ARG, "systems of a batch must share dim");
    if (sys[i]->precision != sys[0]->precision)
      return fail(EWALD_E_ARG, "systems of a batch must share precision");
  }
  for (int w = 0; w < n_walkers; ++w)
    if (walker_sys[w] < 0 || walker_sys[w] >= n_sys) return fail(EWALD_E_ARG, "walker_sys out of range");
  int device = 0;
  int rc = dev_current(&device);
  if (rc) return fail(EWALD_E_HIP, std::string("no HIP device: ") + dev_error_string(rc));
  for (int i = 0; i < n_sys; ++i) {
    ewald_status st = upload_sys(sys[i], device);
    if (st != EWALD_OK) return st;
  }
  std::unique_ptr<ewald_batch> B(new ewald_batch());
  B->sys.assign(sys, sys + n_sys);
  B->walker_sys.assign(walker_sys, walker_sys + n_walkers);
  const int dim = sys[0]->dim;
  B->pos_offsets.assign(size_t(n_walkers) + 1, 0);
  size_t off = 0;
  for (int w = 0; w < n_walkers; ++w) {
    const ewald_sys* s = sys[walker_sys[w]];
    DevWalker dw;
    dw.sys = walker_sys[w];
    dw.n_mobile = s->n_mobile;
    dw.state_off = (long long)off;
    dw.pos_off = (long long)B->pos_offsets[w];
    dw.id = w;
    dw.pad_ = 0;
    B->walkers.push_back(dw);
    B->pos_offsets[w + 1] = B->pos_offsets[w] + size_t(s->n_mobile);
    off += walker_state_bytes(s->n_mobile, dim, s->n_seg, s->dev.n_layers);
  }
  B->state_bytes = off;
  std::vector<DevSys> ds;
  LaunchBatch& L = B->lb;
  if (dev_cu_count(&L.n_cu) != 0 || L.n_cu < 1) L.n_cu = 1;
  L.all_wtab_lds = 1;
  L.all_ortho = 1;
  L.n_walkers = n_walkers;
  L.dim = dim;
  L.mixed = sys[0]->precision == EWALD_FP32_MIXED ? 1 : 0;
  for (int i = 0; i < n_sys; ++i) {
    ds.push_back(sys[i]->dev_uploaded);
    L.has_jastrow |= sys[i]->has_jastrow ? 1 : 0;
    L.has_u |= sys[i]->dev.has_u;
    L.layered |= sys[i]->dev.n_layers > 1 ? 1 : 0;
    L.max_n_seg = std::max(L.max_n_seg, sys[i]->n_seg);
    L.max_nm = std::max(L.max_nm, sys[i]->dev.nm);
    L.max_particles = std::max(L.max_particles, sys[i]->n_mobile);
    L.max_fixed = std::max(L.max_fixed, sys[i]->n_fixed);
    L.refresh_every = std::max(L.refresh_every, L.mixed ? sys[i]->refresh_every : 0);
    L.poly_deg = std::max(L.poly_deg, sys[i]->dev.poly_deg);
    L.max_wtab = std::max(L.max_wtab, sys[i]->dev_uploaded.wtab_lds ? sys[i]->dev_uploaded.n_wtab : 0);
    L.all_wtab_lds &= sys[i]->dev_uploaded.wtab_lds;
    L.all_ortho &= sys[i]->dev.ortho;
  }
  rc = dev_alloc(&B->d_sys, ds.size() * sizeof(DevSys));
  if (rc) return fail(EWALD_E_NOMEM, "device allocation failed");
  rc = dev_alloc(&B->d_walk, B->walkers.size() * sizeof(DevWalker));
  if (rc) return fail(EWALD_E_NOMEM, "device allocation failed");
  // launch order: per-move work (slots + pair terms) descending, stable
  std::vector<DevWalker> order = B->walkers;
  std::stable_sort(order.begin(), order.end(), [&](const DevWalker& a, const DevWalker& b) {
    auto cost = [&](const DevWalker& x) {
      const ewald_sys* s = sys[x.sys];
      return double(s->n_seg) * SEG + 2.0 * (s->n_mobile + s->n_fixed);
    };
    return cost(a) > cost(b);
  });
  rc = dev_upload(B->d_sys, ds.data(), ds.size() * sizeof(DevSys));
  if (!rc) rc = dev_upload(B->d_walk, order.data(), order.size() * sizeof(DevWalker));
  if (rc) return fail(EWALD_E_HIP, std::string("upload failed: ") + dev_error_string(rc));
  L.d_sys = static_cast<const DevSys*>(B->d_sys);
  L.d_walk = static_cast<const DevWalker*>(B->d_walk);
  *out = B.release();
  return EWALD_OK;
} catch (const std::bad_alloc&) {
  return fail(EWALD_E_NOMEM, "host allocation failed");
} catch (...) {
  return fail(EWALD_E_ARG, "unexpected error in ewald_batch_create");
}

ewald_status ewald_batch_layout(const ewald_batch* b, size_t* pos_offsets, size_t* state_bytes) {
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  if (pos_offsets) std::copy(b->pos_offsets.begin(), b->pos_offsets.end(), pos_offsets);
  if (state_bytes) *state_bytes = b->state_bytes;
  return EWALD_OK;
}

ewald_status ewald_state_offsets(const ewald_batch* b, int walker, size_t* hdr, size_t* pos,
                                 size_t* rho) {
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  if (walker < 0 || walker >= int(b->walkers.size())) return fail(EWALD_E_ARG, "walker out of range");
  const DevWalker& w = b->walkers[walker];
  const size_t base = size_t(w.state_off);
  if (hdr) *hdr = base;
  if (pos) *pos = base + HDR_BYTES;
  if (rho) *rho = base + HDR_BYTES + walker_pos_bytes(w.n_mobile, b->lb.dim);
  return EWALD_OK;
}

void ewald_batch_destroy(ewald_batch* b) { delete b; }

ewald_status ewald_energy_batch(ewald_batch* b, const double* pos, void* state, double* energy,
                                double* jastrow, void* stream) {
  CallTimer timer("ewald_energy_batch", stream);
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  if (!pos || !state || !energy) return fail(EWALD_E_ARG, "pos, state and energy must be non-NULL");
  int rc = launch_energy(b->lb, pos, static_cast<char*>(state), energy, jastrow, stream);
  if (rc) return launch_status(rc, "energy");
  return check_state(b, state, 0, 1);
}

ewald_status ewald_move_delta_grad_batch(ewald_batch* b, void* state, const int32_t* k, const double* new_pos,
                                         double* delta, double* djastrow, double* jgrad, double* jlap,
                                         void* stream) {
  CallTimer timer(jgrad ? "ewald_move_delta_grad_batch" : "ewald_move_delta_batch", stream);
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  if (!state || !k || !new_pos || !delta) return fail(EWALD_E_ARG, "state, k, new_pos and delta must be non-NULL");
  if ((jgrad == nullptr) != (jlap == nullptr)) return fail(EWALD_E_ARG, "jgrad and jlap must both be given or both NULL");
  if (jgrad && !b->lb.has_jastrow) return fail(EWALD_E_ARG, "Jastrow derivatives need Jastrow coefficients or a u term");
  ewald_status st = check_state(b, state, 1, -1);
  if (st != EWALD_OK) return st;
  int rc = launch_delta(b->lb, static_cast<char*>(state), k, new_pos, delta, djastrow, jgrad, jlap, stream);
  if (rc) return launch_status(rc, "move_delta");
  return check_state(b, state, 0, 2);
}

ewald_status ewald_move_delta_batch(ewald_batch* b, void* state, const int32_t* k,
                                    const double* new_pos, double* delta, double* djastrow,
                                    void* stream) {
  return ewald_move_delta_grad_batch(b, state, k, new_pos, delta, djastrow, nullptr, nullptr, stream);
}

ewald_status ewald_accept_batch(ewald_batch* b, void* state, const uint8_t* accept, void* stream) {
  CallTimer timer("ewald_accept_batch", stream);
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  if (!state || !accept) return fail(EWALD_E_ARG, "state and accept must be non-NULL");
  ewald_status st = check_state(b, state, 2, -1);
  if (st != EWALD_OK) return st;
  int rc = launch_accept(b->lb, static_cast<char*>(state), accept, stream);
  if (rc) return launch_status(rc, "accept");
  return check_state(b, state, 0, 1);
}

ewald_status ewald_step_batch(ewald_batch* b, void* state, const uint8_t* accept_prev, const int32_t* k,
                              const double* new_pos, double* delta, double* djastrow, double* jgrad, double* jlap,
                              void* stream) {
  CallTimer timer("ewald_step_batch", stream);
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  if (!state || !k || !new_pos || !delta) return fail(EWALD_E_ARG, "state, k, new_pos and delta must be non-NULL");
  if ((jgrad == nullptr) != (jlap == nullptr)) return fail(EWALD_E_ARG, "jgrad and jlap must both be given or both NULL");
  if (jgrad && !b->lb.has_jastrow) return fail(EWALD_E_ARG, "Jastrow derivatives need Jastrow coefficients or a u term");
  ewald_status st = check_state(b, state, accept_prev ? 2 : 1, -1);
  if (st != EWALD_OK) return st;
  int rc = launch_step(b->lb, static_cast<char*>(state), accept_prev, k, new_pos, delta, djastrow, jgrad, jlap,
                       stream);
  if (rc) return launch_status(rc, "step");
  return check_state(b, state, 0, 2);
}

ewald_status ewald_run_moves_grad_batch(ewald_batch* b, void* state, int n_steps, const int32_t* k,
                                        const double* new_pos, const uint8_t* accept, double* delta,
                                        double* djastrow, double* jgrad, double* jlap, void* stream) {
  CallTimer timer(jgrad ? "ewald_run_moves_grad_batch" : "ewald_run_moves_batch", stream);
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  if (n_steps < 0) return fail(EWALD_E_ARG, "n_steps must be >= 0");
  if (!state) return fail(EWALD_E_ARG, "state must be non-NULL");
  if ((jgrad == nullptr) != (jlap == nullptr)) return fail(EWALD_E_ARG, "jgrad and jlap must both be given or both NULL");
  if (jgrad && !b->lb.has_jastrow) return fail(EWALD_E_ARG, "Jastrow derivatives need Jastrow coefficients or a u term");
  ewald_status st = check_state(b, state, 3, -1);
  if (st != EWALD_OK) return st;
  if (n_steps == 0) return EWALD_OK;
  if (!k || !new_pos || !accept || !delta)
    return fail(EWALD_E_ARG, "k, new_pos, accept and delta must be non-NULL");
  int rc = launch_run(b->lb, static_cast<char*>(state), n_steps, k, new_pos, accept, delta, djastrow, jgrad, jlap,
                      stream);
  if (rc) return launch_status(rc, "run_moves");
  return EWALD_OK;
}

ewald_status ewald_run_moves_batch(ewald_batch* b, void* state, int n_steps, const int32_t* k,
                                   const double* new_pos, const uint8_t* accept, double* delta,
                                   double* djastrow, void* stream) {
  return ewald_run_moves_grad_batch(b, state, n_steps, k, new_pos, accept, delta, djastrow, nullptr, nullptr, stream);
}

ewald_status ewald_batch_set_tuning(ewald_batch* b, int threads, int chunk, int general_frame, int waves,
                                    int walkers_per_block) {
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  if (walkers_per_block < 0) return fail(EWALD_E_ARG, "walkers_per_block must be >= 0");
  if (walkers_per_block > 0 && waves > 2)
    return fail(EWALD_E_ARG, "walkers_per_block > 0 runs kernels compiled for two waves per SIMD: waves must be 0 or 2");
  if (!run_threads_valid(b->lb.max_n_seg, threads))
    return fail(EWALD_E_ARG, "threads is not a fused-kernel workgroup size for this batch's segment count");
  if (chunk < 0 || chunk > RUN_CHUNK) return fail(EWALD_E_ARG, "chunk must be in [0, 64]");
  if (general_frame != 0 && general_frame != 1) return fail(EWALD_E_ARG, "general_frame must be 0 or 1");
  if (waves != 0 && waves != 2 && waves != 3 && waves != 4) return fail(EWALD_E_ARG, "waves must be 0, 2, 3 or 4");
  if (waves > 2) {  // the 256-thread kernels come in these variants, and 512 x 2 at four waves
    LaunchBatch L = b->lb;
    L.run_threads = threads;
    RunPlan p{};
    plan_run(L, &p);
    const bool ok = p.threads == 256 || (waves == 4 && p.threads == 512 && p.spt == 2);
    if (!ok)
      return fail(EWALD_E_ARG, "waves 3 and 4 apply to 256-thread workgroups (and 4 to 512 x 2 segments) only");
  }
  std::lock_guard<std::mutex> lk(b->mu);
  b->lb.run_threads = threads;
  b->lb.run_chunk = chunk;
  b->lb.general_frame = general_frame;
  b->lb.run_waves = waves;
  b->lb.run_wpb = walkers_per_block;
  return EWALD_OK;
}

ewald_status ewald_batch_get_tuning(ewald_batch* b, int* threads, int* chunk, int* general_frame,
                                    int* fused, int* waves, int* walkers_per_block) {
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  RunPlan p{};
  {
    std::lock_guard<std::mutex> lk(b->mu);
    plan_run(b->lb, &p);
  }
  if (threads) *threads = p.threads;
  if (chunk) *chunk = p.chunk;
  if (general_frame) *general_frame = p.fused ? p.general_frame : 1;
  if (fused) *fused = p.fused;
  if (waves) *waves = p.fused ? p.waves : 0;
  if (walkers_per_block) *walkers_per_block = p.fused ? p.walkers_per_block : 0;
  return EWALD_OK;
}

namespace {

// Cache key of a tuning: everything the fused kernel's shape depends on.
std::string tune_key(const ewald_batch* b) {
  char arch[128] = "unknown";
  dev_arch(arch, sizeof(arch));
  const LaunchBatch& L = b->lb;
  char buf[512];
  std::snprintf(buf, sizeof(buf), "arch=%s dim=%d mixed=%d jastrow=%d u=%d segs=%d nm=%d particles=%d fixed=%d "
                "poly=%d wtab=%d ortho=%d walkers=%d", arch, L.dim, L.mixed, L.has_jastrow, L.has_u, L.max_n_seg, L.max_nm,
                L.max_particles, L.max_fixed, L.poly_deg, L.max_wtab, L.all_ortho, L.n_walkers);
  return buf;
}

bool cache_lookup(const char* path, const std::string& key, int* t, int* c, int* g, int* v, int* q) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    std::string l(line);
    const size_t bar = l.find('|');
    if (bar == std::string::npos || l.substr(0, bar) != key) continue;
    *q = 0;  // lines written before the queue mode existed have no walkers_per_block
    found = std::sscanf(l.c_str() + bar + 1, "threads=%d chunk=%d general_frame=%d waves=%d walkers_per_block=%d", t,
                        c, g, v, q) >= 4;
  }
  std::fclose(f);
  return found;
}

}  // namespace

ewald_status ewald_autotune(ewald_batch* b, void* state, int n_moves, const char* cache_path, void* stream) {
  CallTimer timer("ewald_autotune", stream);
  if (!b) return fail(EWALD_E_ARG, "batch is NULL");
  if (!state) return fail(EWALD_E_ARG, "state must be non-NULL");
  if (n_moves < 1 || n_moves > 4096) return fail(EWALD_E_ARG, "n_moves must be in [1, 4096]");
  ewald_status st = check_state(b, state, 3, -1);
  if (st != EWALD_OK) return st;
  const std::string key = tune_key(b);
  int t = 0, c = 0, g = 0, v = 0, q = 0;
  // a cached tuning that this library rejects (an edited file, or one from
  // another build) is measured afresh, and the new choice appended
  if (cache_path && cache_lookup(cache_path, key, &t, &c, &g, &v, &q) &&
      ewald_batch_set_tuning(b, t, c, g, v, q) == EWALD_OK)
    return EWALD_OK;
  // probe: proposals spread over each cell, every other move accepted, run on
  // a copy of the walkers' state (which is left as it was)
  const int W = b->lb.n_walkers, dim = b->lb.dim;
  std::vector<uint8_t> ha(size_t(n_moves) * W);
  for (int m = 0; m < n_moves; ++m)
    for (int w = 0; w < W; ++w) ha[size_t(m) * W + w] = uint8_t(m & 1);
  std::vector<int32_t> hk(size_t(n_moves) * W);
  std::vector<double> hp(size_t(n_moves) * W * dim);
  for (int m = 0; m < n_moves; ++m)
    for (int w = 0; w < W; ++w) {
      const ewald_sys* s = b->sys[size_t(b->walker_sys[w])];
      const size_t i = size_t(m) * W + w;
      hk[i] = int32_t((size_t(m) * 7919u + size_t(w) * 104729u) % size_t(s->n_mobile));
      double f[3];  // fractional coordinates spread over the cell
      for (int e = 0; e < dim; ++e)
        f[e] = std::fmod(0.6180339887 * double(m + 1) + 0.4142135624 * double(e + 1) + 0.7320508076 * double(w % 97),
                         1.0);
      for (int d = 0; d < dim; ++d) {
        double x = 0;
        for (int e = 0; e < dim; ++e) x += f[e] * s->dev.A[e * 3 + d];
        hp[i * dim + d] = x;
      }
    }
  void *dk = nullptr, *dp = nullptr, *da = nullptr, *dd = nullptr, *ds = nullptr;
  auto release = [&]() {
    for (void* p : {dk, dp, da, dd, ds})
      if (p) dev_free(p);
  };
  // the caller's stream may still be writing the state (a non-blocking
  // stream does not order against the synchronous copy below)
  int rc = stream_sync(stream);
  if (!rc) rc = dev_alloc(&ds, b->state_bytes);
  if (!rc) rc = dev_copy(ds, state, b->state_bytes);
  if (!rc) rc = dev_alloc(&dk, hk.size() * 4);
  if (!rc) rc = dev_alloc(&dp, hp.size() * 8);
  if (!rc) rc = dev_alloc(&da, size_t(n_moves) * W);
  if (!rc) rc = dev_alloc(&dd, size_t(n_moves) * W * 8);
  if (!rc) rc = dev_upload(dk, hk.data(), hk.size() * 4);
  if (!rc) rc = dev_upload(dp, hp.data(), hp.size() * 8);
  if (!rc) rc = dev_upload(da, ha.data(), ha.size());
  if (rc) {
    release();
    return launch_status(rc, "autotune set-up");
  }
  // candidates: every workgroup shape for the segment count, chunk sizes, both frames
  struct Cand {
    int threads, chunk, general, waves, wpb;
    float ms;
  };
  std::vector<Cand> cands;
  const LaunchBatch saved = b->lb;
  auto probe = [&](Cand& c, int reps) {
    LaunchBatch L = saved;
    L.run_threads = c.threads;
    L.run_chunk = c.chunk;
    L.general_frame = c.general;
    L.run_waves = c.waves;
    L.run_wpb = c.wpb;
    float ms = 0.f;
    const int r = time_run(L, static_cast<char*>(ds), n_moves, static_cast<int32_t*>(dk), static_cast<double*>(dp),
                           static_cast<uint8_t*>(da), static_cast<double*>(dd), stream, reps, &ms);
    if (!r && (c.ms < 0.f || ms < c.ms)) c.ms = ms;
    return r;
  };
  for (int threads : {256, 512, 1024}) {
    if (!run_threads_valid(b->lb.max_n_seg, threads)) continue;
    for (int waves : {2, 3, 4})
    for (int chunk : {0, 32, 16})
      for (int general : {0, 1}) {
        if (general == 0 && !b->lb.all_ortho) continue;
        LaunchBatch L = saved;
        L.run_threads = threads;
        L.run_chunk = chunk;
        L.general_frame = general;
        L.run_waves = waves;
        RunPlan p{};
        plan_run(L, &p);
        if (!p.fused || p.waves != (waves == 2 ? (p.threads <= 512 ? 2 : 0) : waves)) continue;  // no such variant
        cands.push_back({threads, chunk, general, waves, 0, -1.f});
        rc = probe(cands.back(), 2);
        if (rc) {
          release();
          return launch_status(rc, "autotune");
        }
      }
  }
  // second pass: the candidates within 8% of the fastest are timed again,
  // interleaved, and each keeps its best time, so that one noisy probe does
  // not decide between shapes that are close
  auto by_time = [](const Cand& x, const Cand& y) { return x.ms < y.ms; };
  std::stable_sort(cands.begin(), cands.end(), by_time);
  size_t n_close = 0;
  while (n_close < cands.size() && n_close < 4 && cands[n_close].ms <= 1.08f * cands[0].ms) ++n_close;
  for (int pass = 0; pass < 2 && n_close > 1; ++pass)
    for (size_t i = 0; i < n_close; ++i) {
      rc = probe(cands[i], 2);
      if (rc) {
        release();
        return launch_status(rc, "autotune");
      }
    }
  std::stable_sort(cands.begin(), cands.begin() + n_close, by_time);
  // walkers per workgroup: for the chosen shape, a queue (1 walker per
  // workgroup on average, and as many walkers per workgroup as leave one
  // workgroup per slot the device holds at once, when that is more) against
  // the hardware's dispatch of one workgroup per walker, interleaved, each
  // timed three times
  if (!cands.empty()) {
    Cand hw = cands[0];
    hw.ms = -1.f;  // timed afresh, as many times as each queue setting
    LaunchBatch L = saved;
    L.run_threads = hw.threads;
    L.run_chunk = hw.chunk;
    L.general_frame = hw.general;
    L.run_waves = 2;  // the queue mode's kernels are compiled for two waves per SIMD
    RunPlan p{};
    plan_run(L, &p);
    if (p.fused) {
      const int resident = std::max(1, p.blocks_per_cu) * std::max(1, saved.n_cu);
      std::vector<Cand> qs;
      for (int wpb : {1, (W + resident - 1) / resident}) {
        if (!qs.empty() && qs.back().wpb == wpb) continue;
        Cand qc = hw;
        qc.waves = 2;
        qc.wpb = wpb;
        qc.ms = -1.f;
        qs.push_back(qc);
      }
      for (int pass = 0; pass < 3 && !rc; ++pass) {
        rc = probe(hw, 1);
        for (Cand& qc : qs)
          if (!rc) rc = probe(qc, 1);
      }
      if (rc) {
        release();
        return launch_status(rc, "autotune");
      }
      cands[0] = hw;
      for (const Cand& qc : qs)
        if (qc.ms >= 0.f && qc.ms < cands[0].ms) cands[0] = qc;
    }
  }
  const float best = cands.empty() ? -1.f : cands[0].ms;
  const int bt = cands.empty() ? 0 : cands[0].threads, bc = cands.empty() ? 0 : cands[0].chunk,
            bg = cands.empty() ? 0 : cands[0].general, bv = cands.empty() ? 0 : cands[0].waves,
            bq = cands.empty() ? 0 : cands[0].wpb;
  release();
  if (best < 0.f) return EWALD_OK;  // the fused kernel does not fit: nothing to tune
  st = ewald_batch_set_tuning(b, bt, bc, bg, bv, bq);
  if (st != EWALD_OK || !cache_path) return st;
  if (FILE* f = std::fopen(cache_path, "a")) {
    std::fprintf(f, "%s|threads=%d chunk=%d general_frame=%d waves=%d walkers_per_block=%d ms=%.4f\n", key.c_str(),
                 bt, bc, bg, bv, bq, double(best));
    std::fclose(f);
  }
  return EWALD_OK;
}

}  // extern "C"
