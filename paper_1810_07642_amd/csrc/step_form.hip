// The fused step kernels of one storage form and collision stage: the build
// compiles this file once per pair, with STEP_FORM (kF64, kF32 or kF16S) and
// STEP_W1 (0: the general stages, 1: omega = 1) set, so that the pairs
// compile in parallel.
#include "step.h"

namespace tflbm {

template hipError_t launch_step_form<STEP_FORM, STEP_W1 != 0>(int, const StepArgs &, int, bool, hipStream_t);
template int step_occupancy_form<STEP_FORM, STEP_W1 != 0>(int, int, bool);

}  // namespace tflbm
