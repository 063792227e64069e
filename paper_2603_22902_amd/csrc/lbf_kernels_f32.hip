// float32 instantiation of the kernels (populations and most arithmetic in
// float32; enthalpy inversion, rho H and the rest enthalpy population in
// float64).
#include "lbf_adjoint_kernels.h"
#include "lbf_batch.h"
#include "lbf_batch_adjoint.h"
#include "lbf_kernels.h"
#include "lbf_ops.h"

// The moments-pass kernels are instantiated in lbf_kernels_f32_moments.hip,
// which is built with another instruction scheduling strategy.
#define LBF_MOMENT_KERNEL_F32_EXTERN(DIM, NP)                                                   \
  extern template __global__ void lbf::moment_kernel<lbf::CfgOf<DIM, NP, float, float>>(         \
      const float* __restrict__, const float* __restrict__, float* __restrict__,                  \
      lbf::StepArgs<float>, const lbf::KParams* __restrict__);

LBF_MOMENT_KERNEL_F32_EXTERN(2, 1)
LBF_MOMENT_KERNEL_F32_EXTERN(2, 2)
LBF_MOMENT_KERNEL_F32_EXTERN(2, 3)
LBF_MOMENT_KERNEL_F32_EXTERN(2, 4)
LBF_MOMENT_KERNEL_F32_EXTERN(3, 1)
LBF_MOMENT_KERNEL_F32_EXTERN(3, 2)
LBF_MOMENT_KERNEL_F32_EXTERN(3, 3)
LBF_MOMENT_KERNEL_F32_EXTERN(3, 4)

LBF_DEFINE_OPS(ops_f32, float, float, 1)
