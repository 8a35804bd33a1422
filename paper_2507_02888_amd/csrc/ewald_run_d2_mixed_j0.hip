// Fused multi-move kernels: 2D, FP32-mixed form, without the Jastrow sum.
#include "ewald_run.h"

namespace ewald {
int run_d2_mixed_j0(const LaunchBatch& b, const RunArgs& a) { return run_entry<2, true, 0>(b, a); }
}  // namespace ewald
