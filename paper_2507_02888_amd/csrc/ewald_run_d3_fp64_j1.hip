// Fused multi-move kernels: 3D, FP64 form, with the Jastrow value.
#include "ewald_run.h"

namespace ewald {
int run_d3_fp64_j1(const LaunchBatch& b, const RunArgs& a) { return run_entry<3, false, 1>(b, a); }
}  // namespace ewald
