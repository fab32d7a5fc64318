// swe_step_f32.hip -- the FP32 surface-deviation instances of the split step,
// in a unit of their own so that they are built with contracted
// multiply-adds (the FP64 instances in swe_step.hip round every product and
// sum as written).
#include "swe_split.hpp"

namespace swe {

template __global__ void k_split<true, false>(StepArgs);
template __global__ void k_split<true, true>(StepArgs);

}  // namespace swe
