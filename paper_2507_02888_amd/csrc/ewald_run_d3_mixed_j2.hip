// Fused multi-move kernels: 3D, FP32-mixed form, with the Jastrow value and its derivatives.
#include "ewald_run.h"

namespace ewald {
int run_d3_mixed_j2(const LaunchBatch& b, const RunArgs& a) { return run_entry<3, true, 2>(b, a); }
}  // namespace ewald
