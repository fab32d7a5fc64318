// swe_batched_f32.hip -- the FP32 surface-deviation instances of the batched
// step kernels, in a unit of their own so that they are built with
// contracted multiply-adds (the FP64 instances in swe_batched.hip round every
// product and sum as written).
#include "swe_batched_kern.hpp"

namespace swe {

template __global__ void k_batched<true, 64, false>(BatchArgs);
template __global__ void k_batched<true, 32, false>(BatchArgs);
template __global__ void k_batched<true, 64, true>(BatchArgs);
template __global__ void k_batched<true, 32, true>(BatchArgs);
template __global__ void k_plain<true, 64, false>(BatchArgs);
template __global__ void k_plain<true, 32, false>(BatchArgs);
template __global__ void k_plain<true, 64, true>(BatchArgs);
template __global__ void k_plain<true, 32, true>(BatchArgs);
template __global__ void k_pack<true, false>(BatchArgs);
template __global__ void k_pack<true, true>(BatchArgs);

}  // namespace swe
