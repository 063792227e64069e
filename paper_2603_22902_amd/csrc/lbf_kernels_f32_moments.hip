// float32 moments-pass kernels (moment_kernel), instantiated in a unit of
// their own so that they can be built with the maximum-ILP instruction
// scheduling strategy of the AMDGPU backend: it keeps more of a thread's
// population loads in flight, which shortens this load-bound pass, while the
// same strategy lengthens the register-bound collide pass of the main float32
// unit.  That unit declares these instantiations extern.
#include "lbf_kernels.h"

#define LBF_MOMENT_KERNEL_F32(DIM, NP)                                                          \
  template __global__ void lbf::moment_kernel<lbf::CfgOf<DIM, NP, float, float>>(                \
      const float* __restrict__, const float* __restrict__, float* __restrict__,                  \
      lbf::StepArgs<float>, const lbf::KParams* __restrict__);

LBF_MOMENT_KERNEL_F32(2, 1)
LBF_MOMENT_KERNEL_F32(2, 2)
LBF_MOMENT_KERNEL_F32(2, 3)
LBF_MOMENT_KERNEL_F32(2, 4)
LBF_MOMENT_KERNEL_F32(3, 1)
LBF_MOMENT_KERNEL_F32(3, 2)
LBF_MOMENT_KERNEL_F32(3, 3)
LBF_MOMENT_KERNEL_F32(3, 4)
