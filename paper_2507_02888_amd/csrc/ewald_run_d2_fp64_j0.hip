// Fused multi-move kernels: 2D, FP64 form, without the Jastrow sum.
#include "ewald_run.h"

namespace ewald {
int run_d2_fp64_j0(const LaunchBatch& b, const RunArgs& a) { return run_entry<2, false, 0>(b, a); }
}  // namespace ewald
