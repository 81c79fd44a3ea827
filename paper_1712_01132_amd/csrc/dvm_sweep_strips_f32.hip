// The strip-pipeline sweep (dvm_sweep_strips.h) instantiated for FP32.
#include "dvm_sweep_strips.h"

namespace pdvm {
template hipError_t launch_sweep_strips<float>(const Batch<float> &, hipStream_t, const Scratch &);
}  // namespace pdvm
