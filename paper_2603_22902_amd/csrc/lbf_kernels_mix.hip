// float32 storage with float64 arithmetic: the HBM traffic of the float32
// path with the rounding of float64 arithmetic inside each step.
#include "lbf_adjoint_kernels.h"
#include "lbf_batch.h"
#include "lbf_batch_adjoint.h"
#include "lbf_kernels.h"
#include "lbf_ops.h"

LBF_DEFINE_OPS(ops_mix, float, double, 0)
