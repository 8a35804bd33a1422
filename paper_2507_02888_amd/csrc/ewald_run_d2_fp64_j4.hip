// Fused multi-move kernels: 2D, FP64 form, with the Jastrow value, the two-body u term and their derivatives.
#include "ewald_run.h"

namespace ewald {
int run_d2_fp64_j4(const LaunchBatch& b, const RunArgs& a) { return run_entry<2, false, 4>(b, a); }
}  // namespace ewald
