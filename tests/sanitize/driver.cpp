// CPU driver for the sanitizer build: the FP64 oracle (energy, move sequence,
// Jastrow derivatives) and the library's host set-up (ewald_setup and the
// queries, plus its argument checks) on small cells of every shape the
// workloads use.  Exit status 0 when every call returned what it should.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ewald.h"

extern "C" {
typedef struct {
  int dim;
  double lat[9];
  double alpha, r_cut, g_cut;
  int n_jastrow;
  const double* jastrow_a;
  int n_u;
  int u_c;
  double u_cut;
  const double* u_alpha;
  const int* spin;
  const double* z;
} osys;
int oracle_energy(const osys* s, int n, const double* pos, const double* q, double* parts, double* jastrow);
int oracle_run(const osys* s, int n, int n_mobile, const double* pos0, const double* q, int n_steps,
               const int32_t* k, const double* new_pos, const uint8_t* accept, double* e0, double* j0,
               double* delta, double* djas, double* pos_final, double* jgrad, double* jlap);
int oracle_jastrow_derivs(const osys* s, int n, const double* pos, const double* q, int k, double* grad,
                          double* lap);
int oracle_run_batch(const osys* s, int n_walkers, int n, int n_mobile, const double* pos0, const double* q,
                     int n_steps, const int32_t* k, const double* new_pos, const uint8_t* accept, double* e0,
                     double* j0, double* delta, double* djas, int n_threads);
}

static int failures = 0;
#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++failures;                                                   \
    }                                                               \
  } while (0)

static unsigned long long lcg = 12345;
static double urand() {
  lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
  return double(lcg >> 11) * (1.0 / 9007199254740992.0);
}

struct Cell {
  int dim;
  double lat[3][3];
};

static void run_cell(const Cell& c, int n, int n_ions) {
  const int dim = c.dim;
  double vol = dim == 3 ? std::fabs(c.lat[0][0] * (c.lat[1][1] * c.lat[2][2] - c.lat[1][2] * c.lat[2][1]) -
                                    c.lat[0][1] * (c.lat[1][0] * c.lat[2][2] - c.lat[1][2] * c.lat[2][0]) +
                                    c.lat[0][2] * (c.lat[1][0] * c.lat[2][1] - c.lat[1][1] * c.lat[2][0]))
                        : std::fabs(c.lat[0][0] * c.lat[1][1] - c.lat[0][1] * c.lat[1][0]);
  const double L = std::pow(vol, 1.0 / dim);
  std::vector<double> ja(12);
  for (double& a : ja) a = 0.02 * urand() - 0.01;
  std::vector<double> qm(n, -1.0), qf(n_ions, double(n) / (n_ions > 0 ? n_ions : 1)), fpos(n_ions * dim);
  for (double& x : fpos) x = L * urand();
  // oracle
  osys s{};
  s.dim = dim;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s.lat[3 * i + j] = c.lat[i][j];
  s.alpha = 5.0 / L;
  s.r_cut = 0.4 * L;
  s.g_cut = 4.0 * 2 * M_PI / L;
  s.n_jastrow = int(ja.size());
  s.jastrow_a = ja.data();
  const int nt = n + n_ions;
  // Jastrow u term: two channels of 6 coefficients, C = 3, L_u = r_cut;
  // mobile particles alternate spin labels, ions take no part
  std::vector<double> ua(12);
  for (double& x : ua) x = (urand() - 0.5) * 1e-3;
  std::vector<int> spin(nt, -1);
  for (int i = 0; i < n; ++i) spin[i] = i & 1;
  s.n_u = 6;
  s.u_c = 3;
  s.u_cut = s.r_cut;
  s.u_alpha = ua.data();
  s.spin = spin.data();
  std::vector<double> pos(nt * dim), q(nt);
  for (int i = 0; i < n; ++i) {
    q[i] = qm[i];
    for (int d = 0; d < dim; ++d) pos[i * dim + d] = L * urand();
  }
  for (int i = 0; i < n_ions; ++i) {
    q[n + i] = qf[i];
    for (int d = 0; d < dim; ++d) pos[(n + i) * dim + d] = fpos[i * dim + d];
  }
  double parts[5], jas = 0;
  CHECK(oracle_energy(&s, nt, pos.data(), q.data(), parts, &jas) == 0);
  CHECK(std::isfinite(parts[4]) && std::isfinite(jas));
  const int S = 5;
  std::vector<int32_t> k(S);
  std::vector<double> newp(S * dim), delta(S), djas(S), jg(S * dim), jl(S), pf(nt * dim);
  std::vector<uint8_t> acc(S);
  for (int m = 0; m < S; ++m) {
    k[m] = m % n;
    acc[m] = uint8_t(m & 1);
    for (int d = 0; d < dim; ++d) newp[m * dim + d] = L * (1.4 * urand() - 0.2);
  }
  double e0[5], j0 = 0;
  CHECK(oracle_run(&s, nt, n, pos.data(), q.data(), S, k.data(), newp.data(), acc.data(), e0, &j0, delta.data(),
                   djas.data(), pf.data(), jg.data(), jl.data()) == 0);
  for (int m = 0; m < S; ++m) CHECK(std::isfinite(delta[m]) && std::isfinite(jl[m]));
  double grad[3], lap;
  CHECK(oracle_jastrow_derivs(&s, nt, pos.data(), q.data(), 0, grad, &lap) == 0);
  std::vector<double> e0b(2 * 5), j0b(2), db(S * 2), djb(S * 2);
  std::vector<double> pos2(2 * nt * dim);
  std::memcpy(pos2.data(), pos.data(), sizeof(double) * nt * dim);
  std::memcpy(pos2.data() + nt * dim, pos.data(), sizeof(double) * nt * dim);
  std::vector<int32_t> k2(S * 2);
  std::vector<double> newp2(S * 2 * dim);
  std::vector<uint8_t> acc2(S * 2);
  for (int m = 0; m < S; ++m)
    for (int w = 0; w < 2; ++w) {
      k2[m * 2 + w] = k[m];
      acc2[m * 2 + w] = acc[m];
      for (int d = 0; d < dim; ++d) newp2[(m * 2 + w) * dim + d] = newp[m * dim + d];
    }
  CHECK(oracle_run_batch(&s, 2, nt, n, pos2.data(), q.data(), S, k2.data(), newp2.data(), acc2.data(), e0b.data(),
                         j0b.data(), db.data(), djb.data(), 2) >= 1);
  for (int m = 0; m < S; ++m) CHECK(db[m * 2] == delta[m] && db[m * 2 + 1] == delta[m]);

  // host set-up of the library
  for (int prec = 0; prec < 2; ++prec) {
    ewald_sys_desc d{};
    d.dim = dim;
    std::memcpy(d.lattice, c.lat, sizeof(d.lattice));
    d.n_fixed = n_ions;
    d.fixed_pos = fpos.data();
    d.fixed_q = qf.data();
    d.n_mobile = n;
    d.mobile_q = qm.data();
    d.alpha = s.alpha;
    d.g_cut = s.g_cut;
    d.r_cut = s.r_cut;
    d.precision = prec ? EWALD_FP32_MIXED : EWALD_FP64;
    d.refresh_every = prec ? 8 : 0;
    d.n_jastrow = int(ja.size());
    d.jastrow_a = ja.data();
    d.u_terms = s.n_u;
    d.u_C = s.u_c;
    d.u_cutoff = s.u_cut;
    d.u_alpha = ua.data();
    d.mobile_spin = spin.data();  // the first n labels are the mobile particles'
    ewald_sys* sys = nullptr;
    CHECK(ewald_setup(&d, &sys) == EWALD_OK && sys);
    if (!sys) continue;
    int n_g = 0, n_slots = 0, n_sh = 0, n_cand = 0, idx = -1;
    double r_ins = 0, ec = 0, box[3];
    CHECK(ewald_sys_query(sys, &n_g, &n_slots, &n_sh, &r_ins, &ec) == EWALD_OK);
    CHECK(n_g > 0 && n_slots >= n_g && n_sh > 0 && r_ins >= s.r_cut && std::isfinite(ec));
    std::vector<int32_t> nn(n_slots * 3), sh(n_slots);
    std::vector<double> w(n_slots), jj(n_slots);
    CHECK(ewald_sys_tables(sys, nn.data(), w.data(), jj.data(), sh.data()) == EWALD_OK);
    CHECK(ewald_sys_candidates(sys, &n_cand, nullptr) == EWALD_OK);
    std::vector<double> cand(n_cand * 3 + 1);
    CHECK(ewald_sys_candidates(sys, &n_cand, cand.data()) == EWALD_OK);
    CHECK(ewald_sys_geometry(sys, &idx, box) == EWALD_OK && idx >= 0);
    int ws = 0;
    ewald_batch* b = nullptr;
    CHECK(ewald_batch_create(&sys, 1, &ws, 1, &b) == EWALD_E_HIP && b == nullptr);
    ewald_sys_destroy(sys);
    if (dim == 2) {  // a layered system: two planes, no Jastrow terms; and the oracle's layered energy
      ewald_sys_desc dl = d;
      dl.n_jastrow = 0;
      dl.u_terms = 0;
      dl.n_layers = 2;
      dl.layer_z[0] = 0.0;
      dl.layer_z[1] = 0.8;
      dl.n_mobile_layer0 = n / 2;
      std::vector<int32_t> fl(n_ions, 1);
      dl.fixed_layer = fl.data();
      ewald_sys* ls = nullptr;
      CHECK(ewald_setup(&dl, &ls) == EWALD_OK && ls);
      ewald_sys_destroy(ls);
      dl.n_jastrow = int(ja.size());
      CHECK(ewald_setup(&dl, &ls) == EWALD_E_ARG);
      if (prec == 0) {
        std::vector<double> zz(nt, 0.0);
        for (int i = n / 2; i < nt; ++i) zz[i] = 0.8;
        osys sl = s;
        sl.n_jastrow = 0;
        sl.n_u = 0;
        sl.z = zz.data();
        double pl[5], jl0 = 0;
        CHECK(oracle_energy(&sl, nt, pos.data(), q.data(), pl, &jl0) == 0 && std::isfinite(pl[4]));
        CHECK(oracle_run(&sl, nt, n, pos.data(), q.data(), S, k.data(), newp.data(), acc.data(), e0, &j0,
                         delta.data(), djas.data(), pf.data(), nullptr, nullptr) == 0);
      }
    }
    // argument checks
    d.u_cutoff = 10 * L;
    CHECK(ewald_setup(&d, &sys) == EWALD_E_RCUT);
    d.u_cutoff = s.u_cut;
    d.u_C = 20;
    CHECK(ewald_setup(&d, &sys) == EWALD_E_ARG);
    d.u_C = s.u_c;
    d.r_cut = 10 * L;
    CHECK(ewald_setup(&d, &sys) == EWALD_E_RCUT);
    d.r_cut = s.r_cut;
    d.alpha = -1;
    CHECK(ewald_setup(&d, &sys) == EWALD_E_ARG);
  }
}

int main() {
  const double a = 5.0;
  Cell sc{3, {{a, 0, 0}, {0, a, 0}, {0, 0, a}}};
  Cell fcc{3, {{0, a / 2, a / 2}, {a / 2, 0, a / 2}, {a / 2, a / 2, 0}}};
  Cell bcc{3, {{-a / 2, a / 2, a / 2}, {a / 2, -a / 2, a / 2}, {a / 2, a / 2, -a / 2}}};
  Cell tri{3, {{6.0, 0.3, 0.0}, {0.5, 5.5, 0.2}, {0.1, -0.4, 6.2}}};
  Cell hex{2, {{a, 0, 0}, {a / 2, a * std::sqrt(3.0) / 2, 0}, {0, 0, 1}}};
  run_cell(sc, 9, 0);
  run_cell(fcc, 7, 2);
  run_cell(bcc, 8, 0);
  run_cell(tri, 5, 3);
  run_cell(hex, 10, 0);
  ewald_sys* s = nullptr;
  CHECK(ewald_setup(nullptr, &s) == EWALD_E_ARG);
  CHECK(std::strlen(ewald_last_error()) > 0);
  // per-call timers: bookkeeping of calls that fail before any launch
  CHECK(ewald_timing_enable(1) == EWALD_OK);
  for (int i = 0; i < 3; ++i) CHECK(ewald_energy_batch(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == EWALD_E_ARG);
  CHECK(ewald_accept_batch(nullptr, nullptr, nullptr, nullptr) == EWALD_E_ARG);
  char rep[512];
  CHECK(ewald_timing_report(rep, sizeof rep, 1) == EWALD_OK);
  CHECK(std::strstr(rep, "ewald_energy_batch 3 0 ") != nullptr);
  CHECK(std::strstr(rep, "ewald_accept_batch 1 0 ") != nullptr);
  CHECK(ewald_timing_report(rep, sizeof rep, 0) == EWALD_OK);
  CHECK(std::strstr(rep, "ewald_energy_batch") == nullptr);  // reset
  CHECK(ewald_accept_batch(nullptr, nullptr, nullptr, nullptr) == EWALD_E_ARG);
  char small[8];
  CHECK(ewald_timing_report(small, sizeof small, 0) == EWALD_E_ARG && std::strlen(small) == 7);
  CHECK(ewald_timing_report(nullptr, 4, 0) == EWALD_E_ARG);
  CHECK(ewald_timing_enable(0) == EWALD_OK);
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("sanitizer driver: all checks passed\n");
  return 0;
}
