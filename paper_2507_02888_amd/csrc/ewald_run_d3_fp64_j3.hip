// Fused multi-move kernels: 3D, FP64 form, with the Jastrow value and the two-body u term.
#include "ewald_run.h"

namespace ewald {
int run_d3_fp64_j3(const LaunchBatch& b, const RunArgs& a) { return run_entry<3, false, 3>(b, a); }
}  // namespace ewald
