// float32 kernels built with the maximum-ILP instruction scheduling strategy
// of the AMDGPU backend (see build.py): the 3D moment_kernel, the 2D batched
// batch_moment_kernel and the single-case 2D reverse-step kernels (collide
// reverse, both forms, and the tiled gather).  The strategy keeps more of a
// thread's loads in flight, which shortens these passes, while it lengthens
// the register-bound collide pass, the 2D single-case moments pass and the
// batched reverse passes of the main float32 unit.  That unit declares these
// instantiations extern.
#include "lbf_adjoint_kernels.h"
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

#define LBF_ADJ_TILE_KERNELS_F32(NP)                                                               \
  template __global__ void lbf::adj_collide_tile_kernel<lbf::CfgOf<2, NP, float, float>>(        \
      lbf::AdjArgs<lbf::CfgOf<2, NP, float, float>>, const lbf::KParams* __restrict__,            \
      double* __restrict__, int, int, int, int);                                                  \
  template __global__ void lbf::adj_gather_tile_kernel<lbf::CfgOf<2, NP, float, float>>(         \
      lbf::AdjArgs<lbf::CfgOf<2, NP, float, float>>, const lbf::KParams* __restrict__,            \
      double* __restrict__, int, int, int, int);
#define LBF_ADJ_CELL_KERNEL_F32(NP)                                                                \
  template __global__ void lbf::adj_collide_kernel<lbf::CfgOf<2, NP, float, float>>(             \
      lbf::AdjArgs<lbf::CfgOf<2, NP, float, float>>, const lbf::KParams* __restrict__,            \
      double* __restrict__);

LBF_ADJ_TILE_KERNELS_F32(1)
LBF_ADJ_TILE_KERNELS_F32(2)
LBF_ADJ_TILE_KERNELS_F32(3)
LBF_ADJ_TILE_KERNELS_F32(4)
LBF_ADJ_CELL_KERNEL_F32(1)
LBF_ADJ_CELL_KERNEL_F32(2)
