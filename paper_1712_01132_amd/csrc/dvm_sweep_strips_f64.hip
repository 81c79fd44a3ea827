// The strip-pipeline sweep (dvm_sweep_strips.h) instantiated for FP64.
#include "dvm_sweep_strips.h"

namespace pdvm {
template hipError_t launch_sweep_strips<double>(const Batch<double> &, hipStream_t, const Scratch &);
}  // namespace pdvm
