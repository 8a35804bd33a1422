// Stand-ins for the device half of libewald (ewald_device.hip), so that the
// host set-up (ewald_host.cpp) can be built and run on the CPU under the
// address and undefined-behaviour sanitizers.  Every device call reports
// "no device"; the set-up, queries and argument checks run for real.
#include <cstddef>
#include <cstdint>

#include "ewald_internal.h"

namespace ewald {

namespace {
constexpr int kNoDevice = 100;  // hipErrorNoDevice
}

int launch_energy(const LaunchBatch&, const double*, char*, double*, double*, void*) { return kNoDevice; }
int launch_delta(const LaunchBatch&, char*, const int32_t*, const double*, double*, double*, double*, double*,
                 void*) {
  return kNoDevice;
}
int launch_accept(const LaunchBatch&, char*, const uint8_t*, void*) { return kNoDevice; }
int launch_step(const LaunchBatch&, char*, const uint8_t*, const int32_t*, const double*, double*, double*, double*,
                double*, void*) {
  return kNoDevice;
}
int launch_run(const LaunchBatch&, char*, int, const int32_t*, const double*, const uint8_t*, double*, double*,
               double*, double*, void*) {
  return kNoDevice;
}
void plan_run(const LaunchBatch&, RunPlan* plan) { *plan = RunPlan{}; }
bool run_threads_valid(int, int threads) { return threads == 0; }
int time_run(const LaunchBatch&, char*, int, const int32_t*, const double*, const uint8_t*, double*, void*, int,
             float* best_ms) {
  *best_ms = 0.f;
  return kNoDevice;
}
int dev_alloc(void** p, size_t) {
  *p = nullptr;
  return kNoDevice;
}
int dev_free(void*) { return 0; }
int dev_upload(void*, const void*, size_t) { return kNoDevice; }
int dev_current(int*) { return kNoDevice; }
int dev_cu_count(int* n_cu) {
  *n_cu = 0;
  return kNoDevice;
}
const char* dev_error_string(int) { return "no device (sanitizer build)"; }
int dev_arch(char* buf, int len) {
  if (len > 0) buf[0] = '\0';
  return kNoDevice;
}
int dev_memset(void*, int, size_t) { return kNoDevice; }
int dev_copy(void*, const void*, size_t) { return kNoDevice; }
int stream_sync(void*) { return kNoDevice; }
int event_pair_create(void** pair) {
  *pair = nullptr;
  return kNoDevice;
}
int event_pair_record(void*, int, void*) { return kNoDevice; }
int event_pair_elapsed(void*, float* ms) {
  *ms = 0.f;
  return kNoDevice;
}
void event_pair_destroy(void*) {}
int stream_capturing(void*, int* capturing) {
  *capturing = 0;
  return 0;
}

}  // namespace ewald
