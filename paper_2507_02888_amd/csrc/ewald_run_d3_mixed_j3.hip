// Fused multi-move kernels: 3D, FP32-mixed form, with the Jastrow value and the two-body u term.
#include "ewald_run.h"

namespace ewald {
int run_d3_mixed_j3(const LaunchBatch& b, const RunArgs& a) { return run_entry<3, true, 3>(b, a); }
}  // namespace ewald
