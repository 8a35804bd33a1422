// Fused multi-move kernels: 3D, FP32-mixed form, without the Jastrow sum.
#include "ewald_run.h"

namespace ewald {
int run_d3_mixed_j0(const LaunchBatch& b, const RunArgs& a) { return run_entry<3, true, 0>(b, a); }
}  // namespace ewald
