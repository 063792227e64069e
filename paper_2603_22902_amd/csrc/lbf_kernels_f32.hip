// float32 instantiation of the kernels (populations and most arithmetic in
// float32; enthalpy inversion, rho H and the rest enthalpy population in
// float64).
#include "lbf_adjoint_kernels.h"
#include "lbf_batch.h"
#include "lbf_batch_adjoint.h"
#include "lbf_kernels.h"
#include "lbf_ops.h"

LBF_DEFINE_OPS(ops_f32, float, float, 1)
