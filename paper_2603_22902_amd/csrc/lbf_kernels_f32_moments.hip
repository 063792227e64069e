// float32 moments-pass kernels (the 3D moment_kernel and the 2D batched
// batch_moment_kernel), instantiated in a unit of their own so that they can
// be built with the maximum-ILP instruction scheduling strategy of the AMDGPU
// backend: it keeps all of a thread's population loads in flight, which
// shortens these load-bound passes, while the same strategy lengthens the
// register-bound collide pass (and the 2D single-case moments pass) of the
// main float32 unit.  That unit declares these instantiations extern.
#include "lbf_batch.h"
#include "lbf_kernels.h"

#define LBF_MOMENT_KERNEL_F32(DIM, NP)                                                          \
  template __global__ void lbf::moment_kernel<lbf::CfgOf<DIM, NP, float, float>>(                \
      const float* __restrict__, const float* __restrict__, float* __restrict__,                  \
      lbf::StepArgs<float>, const lbf::KParams* __restrict__);

LBF_MOMENT_KERNEL_F32(3, 1)
LBF_MOMENT_KERNEL_F32(3, 2)
LBF_MOMENT_KERNEL_F32(3, 3)
LBF_MOMENT_KERNEL_F32(3, 4)

#define LBF_BATCH_MOMENT_KERNEL_F32(NP, PACKED, PERSIST)                                          \
  template __global__ void lbf::batch_moment_kernel<lbf::CfgOf<2, NP, float, float>, PACKED, PERSIST>( \
      const lbf::BatchCase<float>* __restrict__, int, int, int, const char* __restrict__,         \
      char* __restrict__);
#define LBF_BATCH_MOMENT_KERNELS_F32(NP)          \
  LBF_BATCH_MOMENT_KERNEL_F32(NP, false, false)   \
  LBF_BATCH_MOMENT_KERNEL_F32(NP, false, true)    \
  LBF_BATCH_MOMENT_KERNEL_F32(NP, true, false)    \
  LBF_BATCH_MOMENT_KERNEL_F32(NP, true, true)

LBF_BATCH_MOMENT_KERNELS_F32(1)
LBF_BATCH_MOMENT_KERNELS_F32(2)
LBF_BATCH_MOMENT_KERNELS_F32(3)
LBF_BATCH_MOMENT_KERNELS_F32(4)
