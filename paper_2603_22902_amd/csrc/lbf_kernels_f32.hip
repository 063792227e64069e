// float32 instantiation of the kernels (populations and most arithmetic in
// float32; enthalpy inversion, rho H and the rest enthalpy population in
// float64).
#include "lbf_adjoint_kernels.h"
#include "lbf_batch.h"
#include "lbf_batch_adjoint.h"
#include "lbf_kernels.h"
#include "lbf_ops.h"

// The 3D moments-pass kernels, the batched (2D) ones and the single-case
// reverse-step kernels below are instantiated in lbf_kernels_f32_ilp.hip,
// which is built with another instruction scheduling strategy.
#define LBF_MOMENT_KERNEL_F32_EXTERN(DIM, NP)                                                   \
  extern template __global__ void lbf::moment_kernel<lbf::CfgOf<DIM, NP, float, float>>(         \
      const float* __restrict__, const float* __restrict__, float* __restrict__,                  \
      lbf::StepArgs<float>, const lbf::KParams* __restrict__);

LBF_MOMENT_KERNEL_F32_EXTERN(3, 1)
LBF_MOMENT_KERNEL_F32_EXTERN(3, 2)
LBF_MOMENT_KERNEL_F32_EXTERN(3, 3)
LBF_MOMENT_KERNEL_F32_EXTERN(3, 4)

#define LBF_BATCH_MOMENT_KERNEL_F32_EXTERN(NP, PACKED, PERSIST)                                   \
  extern template __global__ void                                                                 \
  lbf::batch_moment_kernel<lbf::CfgOf<2, NP, float, float>, PACKED, PERSIST>(                     \
      const lbf::BatchCase<float>* __restrict__, int, int, int, const char* __restrict__,         \
      char* __restrict__);
#define LBF_BATCH_MOMENT_KERNELS_F32_EXTERN(NP)        \
  LBF_BATCH_MOMENT_KERNEL_F32_EXTERN(NP, false, false) \
  LBF_BATCH_MOMENT_KERNEL_F32_EXTERN(NP, false, true)  \
  LBF_BATCH_MOMENT_KERNEL_F32_EXTERN(NP, true, false)  \
  LBF_BATCH_MOMENT_KERNEL_F32_EXTERN(NP, true, true)

LBF_BATCH_MOMENT_KERNELS_F32_EXTERN(1)
LBF_BATCH_MOMENT_KERNELS_F32_EXTERN(2)
LBF_BATCH_MOMENT_KERNELS_F32_EXTERN(3)
LBF_BATCH_MOMENT_KERNELS_F32_EXTERN(4)

#define LBF_ADJ_TILE_KERNELS_F32_EXTERN(NP)                                                        \
  extern template __global__ void lbf::adj_collide_tile_kernel<lbf::CfgOf<2, NP, float, float>>( \
      lbf::AdjArgs<lbf::CfgOf<2, NP, float, float>>, const lbf::KParams* __restrict__,            \
      double* __restrict__, int, int, int, int);                                                  \
  extern template __global__ void lbf::adj_gather_tile_kernel<lbf::CfgOf<2, NP, float, float>>(  \
      lbf::AdjArgs<lbf::CfgOf<2, NP, float, float>>, const lbf::KParams* __restrict__,            \
      double* __restrict__, int, int, int, int);
#define LBF_ADJ_CELL_KERNEL_F32_EXTERN(NP)                                                         \
  extern template __global__ void lbf::adj_collide_kernel<lbf::CfgOf<2, NP, float, float>>(      \
      lbf::AdjArgs<lbf::CfgOf<2, NP, float, float>>, const lbf::KParams* __restrict__,            \
      double* __restrict__);

LBF_ADJ_TILE_KERNELS_F32_EXTERN(1)
LBF_ADJ_TILE_KERNELS_F32_EXTERN(2)
LBF_ADJ_TILE_KERNELS_F32_EXTERN(3)
LBF_ADJ_TILE_KERNELS_F32_EXTERN(4)
LBF_ADJ_CELL_KERNEL_F32_EXTERN(1)
LBF_ADJ_CELL_KERNEL_F32_EXTERN(2)

LBF_DEFINE_OPS(ops_f32, float, float, 1)
