// float64 instantiation of the kernels, compiled without floating-point
// contraction so that each operation rounds as written.
#include "lbf_adjoint_kernels.h"
#include "lbf_batch.h"
#include "lbf_batch_adjoint.h"
#include "lbf_kernels.h"
#include "lbf_ops.h"

LBF_DEFINE_OPS(ops_f64, double, double, 1)
