/* A C caller of libewald (no Python, no PyTorch): one unit charge per simple
 * cubic cell in a neutralising background (the Wigner lattice at r_s = 1).
 * With alpha = 7/L no image lies within the cutoff, so the energy is the
 * converged Madelung energy, -0.8800595 Ha (Coldwell-Horsfall and
 * Maradudin, 1960: -1.760119 Ry per r_s).  Moving the lone charge changes
 * nothing (translation invariance): its move delta must vanish, through
 * ewald_move_delta_batch + ewald_accept_batch and through ewald_step_batch.
 * Exit status 0 when every check holds.  Built by the package build step;
 * run by the GPU tests. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "ewald.h"

#define CHECK_EW(call)                                                                    \
  do {                                                                                    \
    ewald_status st_ = (call);                                                            \
    if (st_ != EWALD_OK) {                                                                \
      fprintf(stderr, "%s failed: status %d (%s)\n", #call, (int)st_, ewald_last_error()); \
      return 1;                                                                           \
    }                                                                                     \
  } while (0)

#define CHECK_HIP(call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));        \
      return 1;                                                                \
    }                                                                          \
  } while (0)

int main(void) {
  const double pi = 3.14159265358979323846;
  const double L = cbrt(4.0 * pi / 3.0);
  const double alpha = 7.0 / L;
  const double q = -1.0;
  ewald_sys_desc d;
  memset(&d, 0, sizeof d);
  d.dim = 3;
  d.lattice[0][0] = d.lattice[1][1] = d.lattice[2][2] = L;
  d.n_mobile = 1;
  d.mobile_q = &q;
  d.alpha = alpha;
  d.g_cut = 12.5 * alpha;
  d.r_cut = 0.5 * L;
  d.precision = EWALD_FP64;
  ewald_sys* sys = NULL;
  CHECK_EW(ewald_setup(&d, &sys));
  int n_g = 0;
  CHECK_EW(ewald_sys_query(sys, &n_g, NULL, NULL, NULL, NULL));

  int walker_sys = 0;
  ewald_batch* b = NULL;
  CHECK_EW(ewald_batch_create(&sys, 1, &walker_sys, 1, &b));
  size_t state_bytes = 0;
  CHECK_EW(ewald_batch_layout(b, NULL, &state_bytes));

  const double pos_h[3] = {0.1, 0.2, 0.3};
  const double new_h[2][3] = {{0.7, -0.4, 1.1}, {-0.2, 0.05, 0.4}};
  const int32_t k_h = 0;
  const uint8_t acc_h = 1;
  double *pos, *energy, *new_pos, *delta;
  int32_t* k;
  uint8_t* accept;
  void* state;
  CHECK_HIP(hipMalloc((void**)&pos, sizeof pos_h));
  CHECK_HIP(hipMalloc((void**)&new_pos, sizeof new_h));
  CHECK_HIP(hipMalloc((void**)&energy, sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&delta, 3 * sizeof(double)));
  CHECK_HIP(hipMalloc((void**)&k, sizeof k_h));
  CHECK_HIP(hipMalloc((void**)&accept, sizeof acc_h));
  CHECK_HIP(hipMalloc(&state, state_bytes));
  CHECK_HIP(hipMemcpy(pos, pos_h, sizeof pos_h, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(new_pos, new_h, sizeof new_h, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(k, &k_h, sizeof k_h, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(accept, &acc_h, sizeof acc_h, hipMemcpyHostToDevice));

  CHECK_EW(ewald_energy_batch(b, pos, state, energy, NULL, NULL));
  CHECK_EW(ewald_move_delta_batch(b, state, k, new_pos, delta, NULL, NULL));
  CHECK_EW(ewald_accept_batch(b, state, accept, NULL));
  CHECK_EW(ewald_step_batch(b, state, NULL, k, new_pos + 3, delta + 1, NULL, NULL, NULL, NULL));
  CHECK_EW(ewald_step_batch(b, state, accept, k, new_pos, delta + 2, NULL, NULL, NULL, NULL));
  CHECK_EW(ewald_accept_batch(b, state, accept, NULL));
  CHECK_HIP(hipDeviceSynchronize());

  double e = 0.0, dl[3] = {0.0, 0.0, 0.0};
  CHECK_HIP(hipMemcpy(&e, energy, sizeof e, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(dl, delta, sizeof dl, hipMemcpyDeviceToHost));
  const double ref = -0.8800595;
  int ok = fabs(e - ref) <= 2e-6 * fabs(ref);
  for (int i = 0; i < 3; ++i) ok = ok && fabs(dl[i]) <= 1e-10;
  printf("n_g %d energy %.10f (Madelung %.7f) deltas %.3e %.3e %.3e: %s\n", n_g, e, ref, dl[0], dl[1], dl[2],
         ok ? "ok" : "FAILED");

  hipFree(pos);
  hipFree(new_pos);
  hipFree(energy);
  hipFree(delta);
  hipFree(k);
  hipFree(accept);
  hipFree(state);
  ewald_batch_destroy(b);
  ewald_sys_destroy(sys);
  return ok ? 0 : 2;
}
