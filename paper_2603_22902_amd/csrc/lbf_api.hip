// C ABI of the coupled LB freezing solver (include/lbfreeze.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbfreeze.h"
#include "lbf_adjoint.h"
#include "lbf_batch.h"
#include "lbf_batch_adjoint.h"
#include "lbf_host.h"
#include "lbf_ops.h"

struct lbf_ctx {
  lbf_params prm;
  lbf::KParams kp;
  lbf::Layout lay;
  const lbf::Ops* ops;
  int Q, nlat, naux, dim, N;
  long long ncell;
  char* base;
  hipStream_t stream;
  int device;
  int cur;  // buffer index holding the current state
  bool initialized, nan_flag;
  long long steps;
  std::string err;
};

// A batch: the member contexts grouped by phase count; each group's case
// table (BatchCase, storage-type independent layout) lives in the caller's
// device buffer.
struct lbf_batch_group {
  std::vector<lbf_ctx*> ctx;
  std::vector<int> cur0;        // buffer of each case at even batch steps
  std::vector<int> user;        // index of each case in the caller's list
  std::vector<long long> soff;  // offset of each case in a packed batch state
  int variant;                  // row tile BATCH_TILES[variant]
  int cblocks, mblocks;         // grid sizes of the two passes
  size_t off;                   // case table offset in the device buffer
};

struct lbf_batch {
  lbf_ctx* first;
  int ncase;
  size_t state_bytes;  // packed batch state: the cases' device states in caller order
  lbf_batch_group g[lbf::MAXP];
  char* base;
  hipStream_t stream;
  int parity;  // batch steps taken mod 2
  hipGraph_t graph;
  hipGraphExec_t exec;
  int graph_parity;
  char* own_base;                 // lowest address of the members' state buffers (table offsets)
  unsigned launch;                // LBF_BATCH_PERSISTENT | LBF_BATCH_CONCURRENT
  int grid;                       // persistent blocks per pass (0: the resident count)
  hipStream_t side[lbf::MAXP];    // streams of the groups after the first (concurrent launch)
  hipEvent_t fork, join[lbf::MAXP];
};

struct lbf_adj {
  lbf_ctx* c;
  lbf::AdjBufLayout lay;
  char* base;
  hipStream_t stream;  // the context's stream, or the batch's for a batched sweep
  int cur;             // adjoint buffer holding the adjoint of the current time level
  bool seeded;
  double J;
};

namespace {

static_assert(lbf::NPAR == 22, "the adjoint buffer layout reserves 22 gradient slots");

// out[k] = sum over rows b of part[b][k], one 256-thread block per k: each
// thread sums a strided set of rows in order, then a fixed-shape tree.
__global__ void __launch_bounds__(256) adj_reduce_kernel(const double* __restrict__ part, int nrows, int nv,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nrows; b += 256) s += part[(long long)b * nv + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = red[0];
}

__global__ void adj_zero_kernel(double* __restrict__ x, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) x[k] = 0.0;
}

constexpr uint64_t kSnapMagic = 0x315A4545524642ULL;  // "BFREEZ1"

struct SnapHeader {
  uint64_t magic;
  int32_t dim, nx, ny, nz, nphase, precision;
  uint64_t pop_bytes, aux_bytes;
  int64_t steps;
};

lbf_status fail(lbf_ctx* c, lbf_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

lbf_status hip_fail(lbf_ctx* c, hipError_t e, const char* what) {
  return fail(c, LBF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr, what)                 \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return hip_fail(c, e_, what); \
  } while (0)

void* pop_ptr(lbf_ctx* c, int k) { return c->base + c->lay.off_pop[k]; }
void* aux_ptr(lbf_ctx* c, int k) { return c->base + c->lay.off_aux[k]; }
double* stage_ptr(lbf_ctx* c) { return reinterpret_cast<double*>(c->base + c->lay.off_stage); }
const lbf::KParams* kp_ptr(lbf_ctx* c) { return reinterpret_cast<const lbf::KParams*>(c->base + c->lay.off_kp); }

using lbf::all_finite;

// Copy a device array of n stored values (the state's precision) to a
// float64 host array, plane by plane through the staging buffer.
lbf_status read_back(lbf_ctx* c, const void* dev, long long nplanes, double* out) {
  const long long nc = c->ncell;
  if (c->prm.precision == LBF_FP64) {
    HIPCHK(c, hipMemcpyAsync(out, dev, (size_t)nplanes * nc * 8, hipMemcpyDeviceToHost, c->stream),
           "hipMemcpyAsync");
  } else {
    const float* src = static_cast<const float*>(dev);
    for (long long k = 0; k < nplanes; ++k) {
      HIPCHK(c, c->ops->widen(src + k * nc, stage_ptr(c), nc, c->stream), "widen");
      HIPCHK(c, hipMemcpyAsync(out + k * nc, stage_ptr(c), (size_t)nc * 8, hipMemcpyDeviceToHost,
                               c->stream),
             "hipMemcpyAsync");
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return LBF_OK;
}

}  // namespace

extern "C" {

lbf_status lbf_check_params(const lbf_params* prm, char* msg, size_t msg_len) {
  const std::string e = lbf::check_params(prm);
  if (msg && msg_len) {
    strncpy(msg, e.c_str(), msg_len - 1);
    msg[msg_len - 1] = 0;
  }
  return e.empty() ? LBF_OK : LBF_EINVAL;
}

lbf_status lbf_state_bytes(const lbf_params* prm, size_t* bytes) {
  if (!bytes) return LBF_EINVAL;
  if (!lbf::check_params(prm).empty()) return LBF_EINVAL;
  *bytes = lbf::make_layout(prm).total;
  return LBF_OK;
}

lbf_status lbf_create(const lbf_params* prm, void* dev_buf, size_t bytes, void* hip_stream,
                      lbf_ctx** out) {
  if (!out) return LBF_EINVAL;
  *out = nullptr;
  if (!lbf::check_params(prm).empty()) return LBF_EINVAL;
  const lbf::Layout lay = lbf::make_layout(prm);
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) & 255)) return LBF_EINVAL;
  if (bytes < lay.total) return LBF_ENOMEM;
  const lbf::Ops* ops = prm->precision == LBF_FP64   ? lbf::ops_f64(prm->dim, prm->nphase)
                        : prm->precision == LBF_MIXED ? lbf::ops_mix(prm->dim, prm->nphase)
                                                      : lbf::ops_f32(prm->dim, prm->nphase);
  if (!ops) return LBF_ENOTSUP;
  lbf_ctx* c = new (std::nothrow) lbf_ctx();
  if (!c) return LBF_ENOMEM;
  c->prm = *prm;
  if (prm->dim == 2) c->prm.nz = 1;
  c->kp = lbf::make_kparams(&c->prm);
  c->lay = lay;
  c->ops = ops;
  c->dim = prm->dim;
  c->N = prm->nphase;
  c->Q = lbf::lattice_q(prm->dim);
  c->nlat = c->N + 2;
  c->naux = c->N + c->dim + 3;
  c->ncell = c->kp.ncell;
  c->base = static_cast<char*>(dev_buf);
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
  c->cur = 0;
  c->initialized = c->nan_flag = false;
  c->steps = 0;
  if (hipGetDevice(&c->device) != hipSuccess ||
      hipMemcpyAsync(c->base + lay.off_kp, &c->kp, sizeof(c->kp), hipMemcpyHostToDevice, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    delete c;
    return LBF_EDEVICE;
  }
  *out = c;
  return LBF_OK;
}

lbf_status lbf_init_fields(lbf_ctx* c, const double* phi, const double* T, const double* u,
                           const double* p) {
  if (!c) return LBF_EINVAL;
  if (!phi || !T) return fail(c, LBF_EINVAL, "phi and T are required");
  const long long nc = c->ncell;
  const int N = c->N, d = c->dim;
  if (!all_finite(phi, (long long)N * nc) || !all_finite(T, nc) ||
      (u && !all_finite(u, (long long)d * nc)) || (p && !all_finite(p, nc)))
    return fail(c, LBF_EINVAL, "initial fields must be finite");
  for (long long k = 0; k < nc; ++k) {
    double s = 0.0;
    for (int q = 0; q < N; ++q) {
      const double v = phi[(long long)q * nc + k];
      if (v < -1e-12) return fail(c, LBF_EINVAL, "phi_p must be non-negative");
      s += v;
    }
    if (fabs(s - 1.0) > 1e-12) return fail(c, LBF_EINVAL, "sum_p phi_p must equal 1 within 1e-12");
  }
  // Upload into the second population buffer (free until the first step).
  const int scratch = 1 - c->cur;
  double* f = static_cast<double*>(pop_ptr(c, scratch));
  size_t off = 0;
  HIPCHK(c, hipMemcpyAsync(f, phi, (size_t)N * nc * 8, hipMemcpyHostToDevice, c->stream), "upload phi");
  off += (size_t)N * nc;
  HIPCHK(c, hipMemcpyAsync(f + off, T, (size_t)nc * 8, hipMemcpyHostToDevice, c->stream), "upload T");
  off += nc;
  if (u) {
    HIPCHK(c, hipMemcpyAsync(f + off, u, (size_t)d * nc * 8, hipMemcpyHostToDevice, c->stream),
           "upload u");
    off += (size_t)d * nc;
  }
  if (p) HIPCHK(c, hipMemcpyAsync(f + off, p, (size_t)nc * 8, hipMemcpyHostToDevice, c->stream), "upload p");
  const int dst = c->cur;
  HIPCHK(c, c->ops->init(c->kp, kp_ptr(c), f, u ? 1 : 0, p ? 1 : 0, pop_ptr(c, dst), aux_ptr(c, dst), c->stream),
         "init kernel");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  c->initialized = true;
  c->nan_flag = false;
  c->steps = 0;
  c->err.clear();
  return LBF_OK;
}

lbf_status lbf_step(lbf_ctx* c, int nsteps) {
  if (!c) return LBF_EINVAL;
  if (nsteps < 0) return fail(c, LBF_EINVAL, "nsteps must be >= 0");
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  for (int s = 0; s < nsteps; ++s) {
    const int a = c->cur, b = 1 - c->cur;
    HIPCHK(c, c->ops->step(pop_ptr(c, a), pop_ptr(c, b), aux_ptr(c, a), aux_ptr(c, b), nullptr, 0, c->kp,
                           kp_ptr(c), c->stream, false, 3),
           "step kernels");
    c->cur = b;
    ++c->steps;
  }
  return LBF_OK;
}

lbf_status lbf_step_timed(lbf_ctx* c, int nsteps, double* ms) {
  if (!c) return LBF_EINVAL;
  if (!ms) return fail(c, LBF_EINVAL, "ms is NULL");
  if (nsteps < 1 || nsteps > 4096) return fail(c, LBF_EINVAL, "nsteps must be in [1, 4096]");
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  const int ne = 2 * nsteps + 1;
  hipEvent_t* ev = new (std::nothrow) hipEvent_t[ne];
  if (!ev) return fail(c, LBF_ENOMEM, "event table");
  int made = 0;
  hipError_t e = hipSuccess;
  for (; made < ne && e == hipSuccess; ++made) e = hipEventCreate(&ev[made]);
  if (e != hipSuccess) --made;
  const char* what = "hipEventCreate";
  int done = 0;
  if (e == hipSuccess) {
    what = "hipEventRecord";
    e = hipEventRecord(ev[0], c->stream);
    for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
      const int a = c->cur, b = 1 - c->cur;
      what = "moments kernel";
      e = c->ops->step(pop_ptr(c, a), pop_ptr(c, b), aux_ptr(c, a), aux_ptr(c, b), nullptr, 0, c->kp,
                       kp_ptr(c), c->stream, false, 1);
      if (e == hipSuccess) {
        what = "hipEventRecord";
        e = hipEventRecord(ev[2 * s + 1], c->stream);
      }
      if (e == hipSuccess) {
        what = "collide kernel";
        e = c->ops->step(pop_ptr(c, a), pop_ptr(c, b), aux_ptr(c, a), aux_ptr(c, b), nullptr, 0, c->kp,
                         kp_ptr(c), c->stream, false, 2);
      }
      if (e == hipSuccess) {
        what = "hipEventRecord";
        e = hipEventRecord(ev[2 * s + 2], c->stream);
      }
      if (e == hipSuccess) {
        c->cur = b;
        ++c->steps;
        ++done;
      }
    }
  }
  if (e == hipSuccess) {
    what = "hipEventSynchronize";
    e = hipEventSynchronize(ev[ne - 1]);
  }
  double tm = 0.0, tc = 0.0;
  for (int s = 0; s < done && e == hipSuccess; ++s) {
    float t1 = 0.f, t2 = 0.f;
    what = "hipEventElapsedTime";
    e = hipEventElapsedTime(&t1, ev[2 * s], ev[2 * s + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t2, ev[2 * s + 1], ev[2 * s + 2]);
    tm += t1;
    tc += t2;
  }
  for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
  delete[] ev;
  if (e != hipSuccess) return hip_fail(c, e, what);
  ms[0] = tm / nsteps;
  ms[1] = tc / nsteps;
  return LBF_OK;
}

lbf_status lbf_get_moments(lbf_ctx* c, unsigned mask, double* out) {
  if (!c) return LBF_EINVAL;
  if (!out) return fail(c, LBF_EINVAL, "out is NULL");
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  const int N = c->N, d = c->dim;
  const long long nc = c->ncell;
  // field ids: phi_p (0..N-1), rhoH N, T N+1, f_l N+2, rho N+3, u N+4.., p N+4+d, mdot N+5+d
  int ids[16], nf = 0;
  if (mask & LBF_M_PHI)
    for (int q = 0; q < N; ++q) ids[nf++] = q;
  if (mask & LBF_M_RHOH) ids[nf++] = N;
  if (mask & LBF_M_T) ids[nf++] = N + 1;
  if (mask & LBF_M_FL) ids[nf++] = N + 2;
  if (mask & LBF_M_RHO) ids[nf++] = N + 3;
  if (mask & LBF_M_U)
    for (int a = 0; a < d; ++a) ids[nf++] = N + 4 + a;
  if (mask & LBF_M_P) ids[nf++] = N + 4 + d;
  if (mask & LBF_M_MDOT) ids[nf++] = N + 5 + d;
  const int a = c->cur;
  // The other aux buffer is free between steps: the moments pass writes
  // phi_p, f_s there.
  for (int k = 0; k < nf; ++k) {
    HIPCHK(c, c->ops->step(pop_ptr(c, a), nullptr, aux_ptr(c, a), aux_ptr(c, 1 - a), stage_ptr(c), ids[k], c->kp,
                           kp_ptr(c), c->stream, true, 3),
           "moments kernel");
    HIPCHK(c, hipMemcpyAsync(out + (long long)k * nc, stage_ptr(c), (size_t)nc * 8, hipMemcpyDeviceToHost,
                             c->stream),
           "hipMemcpyAsync");
  }
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return LBF_OK;
}

lbf_status lbf_get_populations(lbf_ctx* c, double* out) {
  if (!c) return LBF_EINVAL;
  if (!out) return fail(c, LBF_EINVAL, "out is NULL");
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  return read_back(c, pop_ptr(c, c->cur), (long long)c->nlat * c->Q, out);
}

lbf_status lbf_get_aux(lbf_ctx* c, double* out) {
  if (!c) return LBF_EINVAL;
  if (!out) return fail(c, LBF_EINVAL, "out is NULL");
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  return read_back(c, aux_ptr(c, c->cur), c->naux, out);
}

lbf_status lbf_diagnostics(lbf_ctx* c, double* out) {
  if (!c) return LBF_EINVAL;
  if (!out) return fail(c, LBF_EINVAL, "out is NULL");
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  double* part = reinterpret_cast<double*>(c->base + c->lay.off_part);
  double* dout = reinterpret_cast<double*>(c->base + c->lay.off_out);
  HIPCHK(c, c->ops->diag(c->kp, kp_ptr(c), pop_ptr(c, c->cur), aux_ptr(c, c->cur), part, dout, c->stream),
         "diag kernel");
  HIPCHK(c, hipMemcpyAsync(out, dout, (size_t)c->lay.nv * 8, hipMemcpyDeviceToHost, c->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (out[3 * c->N + 3] != 0.0) c->nan_flag = true;
  if (c->nan_flag) return fail(c, LBF_ENAN, "non-finite order parameter or enthalpy in the state");
  return LBF_OK;
}

// ---------------------------------------------------------------------------
// lbf_diagnostics_noalloc: the same reduction with its per-block partials and
// its result in a file-scope device array instead of the context's buffer.
// Each device holds its own copy of the array; its address is looked up once
// per device (with that device current) and kept, because the array's name
// in host code is not a device address.  Calls that overlap on one device
// share the array and race; every value the kernels read is written earlier
// in the same call, so nothing needs clearing.
// ---------------------------------------------------------------------------
namespace {
static_assert(LBF_DIAG_MAX_BLOCKS == lbf::DIAG_MAX_BLOCKS, "scratch rows = diagnostics blocks");
static_assert(LBF_DIAG_MAX_VALUES >= 3 * lbf::MAXP + 4, "scratch row holds every diagnostic value");
constexpr int kDiagScratchDoubles = LBF_DIAG_MAX_BLOCKS * LBF_DIAG_MAX_VALUES + LBF_DIAG_MAX_VALUES;
static __device__ __align__(256) double scratch[kDiagScratchDoubles];
constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices];  // per device, NULL until looked up
}  // namespace

lbf_status lbf_diagnostics_noalloc(lbf_ctx* c, double* out) {
  if (!c) return LBF_EINVAL;
  if (!out) return fail(c, LBF_EINVAL, "out is NULL");
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  if (c->device < 0 || c->device >= kMaxDevices)
    return fail(c, LBF_ENOTSUP, "device index beyond the static scratch table");
  const int nblocks = lbf::diag_blocks(c->ncell);
  if (nblocks > LBF_DIAG_MAX_BLOCKS || c->lay.nv > LBF_DIAG_MAX_VALUES)
    return fail(c, LBF_EINVAL, "diagnostic partials exceed the static scratch array");
  if (!g_scratch_ptr[c->device]) {
    int prev = -1;
    HIPCHK(c, hipGetDevice(&prev), "hipGetDevice");
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    HIPCHK(c, hipSetDevice(prev), "hipSetDevice");
    HIPCHK(c, e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[c->device] = static_cast<double*>(ptr);
  }
  double* part = g_scratch_ptr[c->device];
  double* dout = part + (size_t)LBF_DIAG_MAX_BLOCKS * LBF_DIAG_MAX_VALUES;
  HIPCHK(c, c->ops->diag(c->kp, kp_ptr(c), pop_ptr(c, c->cur), aux_ptr(c, c->cur), part, dout, c->stream),
         "diag kernel");
  HIPCHK(c, hipMemcpyAsync(out, dout, (size_t)c->lay.nv * 8, hipMemcpyDeviceToHost, c->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (out[3 * c->N + 3] != 0.0) c->nan_flag = true;
  if (c->nan_flag) return fail(c, LBF_ENAN, "non-finite order parameter or enthalpy in the state");
  return LBF_OK;
}

lbf_status lbf_snapshot_bytes(const lbf_ctx* c, size_t* bytes) {
  if (!c || !bytes) return LBF_EINVAL;
  *bytes = sizeof(SnapHeader) + c->lay.pop_bytes + c->lay.aux_bytes;
  return LBF_OK;
}

lbf_status lbf_save_state(lbf_ctx* c, void* host, size_t bytes) {
  if (!c) return LBF_EINVAL;
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  size_t need;
  lbf_snapshot_bytes(c, &need);
  if (!host || bytes != need) return fail(c, LBF_EINVAL, "snapshot buffer has the wrong size");
  SnapHeader h;
  memset(&h, 0, sizeof h);
  h.magic = kSnapMagic;
  h.dim = c->prm.dim;
  h.nx = c->prm.nx;
  h.ny = c->prm.ny;
  h.nz = c->prm.nz;
  h.nphase = c->N;
  h.precision = c->prm.precision;
  h.pop_bytes = c->lay.pop_bytes;
  h.aux_bytes = c->lay.aux_bytes;
  h.steps = c->steps;
  char* dst = static_cast<char*>(host);
  memcpy(dst, &h, sizeof h);
  HIPCHK(c, hipMemcpyAsync(dst + sizeof h, pop_ptr(c, c->cur), c->lay.pop_bytes, hipMemcpyDeviceToHost,
                           c->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipMemcpyAsync(dst + sizeof h + c->lay.pop_bytes, aux_ptr(c, c->cur), c->lay.aux_bytes,
                           hipMemcpyDeviceToHost, c->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return LBF_OK;
}

lbf_status lbf_load_state(lbf_ctx* c, const void* host, size_t bytes) {
  if (!c) return LBF_EINVAL;
  size_t need;
  lbf_snapshot_bytes(c, &need);
  if (!host || bytes != need) return fail(c, LBF_EINVAL, "snapshot has the wrong size");
  SnapHeader h;
  memcpy(&h, host, sizeof h);
  if (h.magic != kSnapMagic || h.dim != c->prm.dim || h.nx != c->prm.nx || h.ny != c->prm.ny ||
      h.nz != c->prm.nz || h.nphase != c->N || h.precision != c->prm.precision ||
      h.pop_bytes != c->lay.pop_bytes || h.aux_bytes != c->lay.aux_bytes || h.steps < 0)
    return fail(c, LBF_EINVAL, "snapshot does not match this context");
  const char* src = static_cast<const char*>(host);
  HIPCHK(c, hipMemcpyAsync(pop_ptr(c, c->cur), src + sizeof h, c->lay.pop_bytes, hipMemcpyHostToDevice,
                           c->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipMemcpyAsync(aux_ptr(c, c->cur), src + sizeof h + c->lay.pop_bytes, c->lay.aux_bytes,
                           hipMemcpyHostToDevice, c->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  c->steps = h.steps;
  c->initialized = true;
  c->nan_flag = false;
  return LBF_OK;
}

lbf_status lbf_state_device_bytes(const lbf_ctx* c, size_t* bytes) {
  if (!c || !bytes) return LBF_EINVAL;
  *bytes = c->lay.pop_bytes + c->lay.aux_bytes;
  return LBF_OK;
}

lbf_status lbf_state_to_device(lbf_ctx* c, void* dst) {
  if (!c) return LBF_EINVAL;
  if (!dst) return fail(c, LBF_EINVAL, "dst is NULL");
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  char* d = static_cast<char*>(dst);
  HIPCHK(c, hipMemcpyAsync(d, pop_ptr(c, c->cur), c->lay.pop_bytes, hipMemcpyDeviceToDevice, c->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipMemcpyAsync(d + c->lay.pop_bytes, aux_ptr(c, c->cur), c->lay.aux_bytes, hipMemcpyDeviceToDevice,
                           c->stream),
         "hipMemcpyAsync");
  return LBF_OK;
}

lbf_status lbf_step_states(lbf_ctx* c, const void* src, void* dst) {
  if (!c) return LBF_EINVAL;
  if (!src || !dst || src == dst) return fail(c, LBF_EINVAL, "src and dst must be distinct device states");
  const char* s = static_cast<const char*>(src);
  char* d = static_cast<char*>(dst);
  HIPCHK(c, c->ops->step(s, d, s + c->lay.pop_bytes, d + c->lay.pop_bytes, nullptr, 0, c->kp, kp_ptr(c),
                         c->stream, false, 3),
         "step kernels");
  return LBF_OK;
}

lbf_status lbf_state_from_device(lbf_ctx* c, const void* src, long long steps) {
  if (!c) return LBF_EINVAL;
  if (!src) return fail(c, LBF_EINVAL, "src is NULL");
  if (steps < 0) return fail(c, LBF_EINVAL, "steps must be >= 0");
  const char* s = static_cast<const char*>(src);
  HIPCHK(c, hipMemcpyAsync(pop_ptr(c, c->cur), s, c->lay.pop_bytes, hipMemcpyDeviceToDevice, c->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipMemcpyAsync(aux_ptr(c, c->cur), s + c->lay.pop_bytes, c->lay.aux_bytes, hipMemcpyDeviceToDevice,
                           c->stream),
         "hipMemcpyAsync");
  c->steps = steps;
  c->initialized = true;
  c->nan_flag = false;
  return LBF_OK;
}

// ----- reverse step ----------------------------------------------------
lbf_status lbf_adjoint_bytes(const lbf_params* prm, size_t* bytes) {
  if (!bytes) return LBF_EINVAL;
  if (!lbf::check_params(prm).empty()) return LBF_EINVAL;
  if (prm->dim != 2 || prm->precision == LBF_MIXED) return LBF_ENOTSUP;
  // the reverse passes address each buffer (population adjoints, lagged-field
  // adjoints, work planes) through a buffer resource of a 31-bit span
  const long long nc = (long long)prm->nx * prm->ny;
  const long long elt = prm->precision == LBF_FP64 ? 8 : 4;
  const long long planes = std::max<long long>((prm->nphase + 2) * 9, lbf::adj_nwork(prm->nphase, 2));
  if (planes * nc * elt >= (1LL << 31)) return LBF_EINVAL;
  *bytes = lbf::make_adj_layout(prm, lbf::make_layout(prm)).total;
  return LBF_OK;
}

lbf_status lbf_adjoint_create(lbf_ctx* c, void* dev_buf, size_t bytes, lbf_adj** out) {
  if (!c || !out) return LBF_EINVAL;
  *out = nullptr;
  if (!c->ops->adjoint) return fail(c, LBF_ENOTSUP, "the reverse step is built for 2D float32 and float64");
  const lbf::AdjBufLayout lay = lbf::make_adj_layout(&c->prm, c->lay);
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) & 255))
    return fail(c, LBF_EINVAL, "adjoint buffer must be 256-byte aligned");
  if (bytes < lay.total) return fail(c, LBF_ENOMEM, "adjoint buffer smaller than lbf_adjoint_bytes");
  lbf_adj* a = new (std::nothrow) lbf_adj();
  if (!a) return LBF_ENOMEM;
  a->c = c;
  a->lay = lay;
  a->base = static_cast<char*>(dev_buf);
  a->stream = c->stream;
  a->cur = 0;
  a->seeded = false;
  a->J = 0.0;
  *out = a;
  return LBF_OK;
}

namespace {
void* adj_lp(lbf_adj* a, int k) { return a->base + a->lay.off_lp[k]; }
void* adj_la(lbf_adj* a, int k) { return a->base + a->lay.off_la[k]; }
void* adj_work(lbf_adj* a) { return a->base + a->lay.off_work; }
// per-block rows of the gradient accumulator (NPAR each), then the objective
// partials (2 per block), the reduced gradient and the objective sums
double* adj_part(lbf_adj* a) { return reinterpret_cast<double*>(a->base + a->lay.off_part); }
double* adj_opart(lbf_adj* a) { return adj_part(a) + (size_t)a->lay.nblocks * lbf::NPAR; }
double* adj_acc(lbf_adj* a) { return reinterpret_cast<double*>(a->base + a->lay.off_acc); }
double* adj_obj(lbf_adj* a) { return reinterpret_cast<double*>(a->base + a->lay.off_obj); }

lbf_status adj_pass(lbf_adj* a, int pass, const void* pin, const void* ain, const void* lpin, const void* lain,
                    void* lpout, void* laout, double A, double B, const void* mom = nullptr) {
  lbf_ctx* c = a->c;
  HIPCHK(c, c->ops->adjoint(pass, pin, ain, lpin, lain, lpout, laout, mom, adj_work(a), c->kp, kp_ptr(c),
                            pass == 4 ? adj_opart(a) : adj_part(a), A, B, a->stream),
         "adjoint kernel");
  return LBF_OK;
}

lbf_status adj_reduce(lbf_adj* a, const double* part, int nv, int nrows, double* out) {
  lbf_ctx* c = a->c;
  hipLaunchKernelGGL(adj_reduce_kernel, dim3(nv), dim3(256), 0, a->stream, part, nrows, nv, out);
  HIPCHK(c, hipGetLastError(), "adjoint reduction");
  return LBF_OK;
}
}  // namespace

#define ADJCHK(expr)                      \
  do {                                    \
    const lbf_status s_ = (expr);         \
    if (s_ != LBF_OK) return s_;          \
  } while (0)

namespace {
// Objective of the state (pin, ain) of a's context; resets the gradient
// rows and sets the adjoint to dJ/dx (buffers 0).
lbf_status adj_seed_at(lbf_adj* a, int objective, const void* pin, const void* ain, double* J) {
  lbf_ctx* c = a->c;
  if (objective != LBF_OBJ_FROZEN_FRACTION && objective != LBF_OBJ_FRONT)
    return fail(c, LBF_EINVAL, "unknown objective");
  ADJCHK(adj_pass(a, 0, pin, ain, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0));
  ADJCHK(adj_pass(a, 4, pin, ain, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0));
  ADJCHK(adj_reduce(a, adj_opart(a), 2, a->lay.cblocks, adj_obj(a)));
  double AB[2];
  HIPCHK(c, hipMemcpyAsync(AB, adj_obj(a), sizeof AB, hipMemcpyDeviceToHost, a->stream), "hipMemcpyAsync");
  HIPCHK(c, hipStreamSynchronize(a->stream), "hipStreamSynchronize");
  if (objective == LBF_OBJ_FROZEN_FRACTION && !(AB[1] > 0.0))
    return fail(c, LBF_EINVAL, "no freezing material in the state (sum psi = 0)");
  // J = A / D: frozen fraction D = sum psi, front position D = cells per
  // wall layer
  const double D = objective == LBF_OBJ_FRONT ? double(c->kp.area) : AB[1];
  const double shift = objective == LBF_OBJ_FRONT ? 0.0 : AB[0] / D;
  const int nz = a->lay.nblocks * lbf::NPAR;
  hipLaunchKernelGGL(adj_zero_kernel, dim3((nz + 255) / 256), dim3(256), 0, a->stream, adj_part(a), nz);
  HIPCHK(c, hipGetLastError(), "adjoint zero");
  ADJCHK(adj_pass(a, 5, pin, ain, nullptr, nullptr, nullptr, nullptr, shift, 1.0 / D));
  ADJCHK(adj_pass(a, 3, pin, ain, nullptr, nullptr, adj_lp(a, 0), adj_la(a, 0), 0.0, 0.0));
  a->cur = 0;
  a->seeded = true;
  a->J = AB[0] / D;
  if (J) *J = a->J;
  return LBF_OK;
}
}  // namespace

lbf_status lbf_adjoint_seed(lbf_adj* a, double* J) { return lbf_adjoint_seed_objective(a, LBF_OBJ_FROZEN_FRACTION, J); }

lbf_status lbf_adjoint_seed_objective(lbf_adj* a, int objective, double* J) {
  if (!a) return LBF_EINVAL;
  lbf_ctx* c = a->c;
  if (!c->initialized) return fail(c, LBF_ESTATE, "lbf_init_fields has not been called");
  return adj_seed_at(a, objective, pop_ptr(c, c->cur), aux_ptr(c, c->cur), J);
}

lbf_status lbf_adjoint_step(lbf_adj* a, const void* state, const void* next) {
  if (!a) return LBF_EINVAL;
  lbf_ctx* c = a->c;
  if (!a->seeded) return fail(c, LBF_ESTATE, "lbf_adjoint_seed has not been called");
  if (!state) return fail(c, LBF_EINVAL, "state is NULL");
  const char* pin = static_cast<const char*>(state);
  const char* ain = pin + c->lay.pop_bytes;
  const char* mom = next ? static_cast<const char*>(next) + c->lay.pop_bytes : nullptr;
  const int k = a->cur;
  if (!mom) ADJCHK(adj_pass(a, 0, pin, ain, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0));
  ADJCHK(adj_pass(a, 1, pin, ain, adj_lp(a, k), adj_la(a, k), adj_lp(a, 1 - k), adj_la(a, 1 - k), 0.0, 0.0, mom));
  ADJCHK(adj_pass(a, 2, pin, ain, adj_lp(a, k), adj_la(a, k), adj_lp(a, 1 - k), adj_la(a, 1 - k), 0.0, 0.0, mom));
  a->cur = 1 - k;
  return LBF_OK;
}

lbf_status lbf_adjoint_finish(lbf_adj* a, const void* state0) {
  if (!a) return LBF_EINVAL;
  lbf_ctx* c = a->c;
  if (!a->seeded) return fail(c, LBF_ESTATE, "lbf_adjoint_seed has not been called");
  if (!state0) return fail(c, LBF_EINVAL, "state0 is NULL");
  const char* pin = static_cast<const char*>(state0);
  const char* ain = pin + c->lay.pop_bytes;
  ADJCHK(adj_pass(a, 6, pin, ain, adj_lp(a, a->cur), adj_la(a, a->cur), nullptr, nullptr, 0.0, 0.0));
  return LBF_OK;
}

lbf_status lbf_adjoint_gradient(lbf_adj* a, double* grad) {
  if (!a) return LBF_EINVAL;
  lbf_ctx* c = a->c;
  if (!grad) return fail(c, LBF_EINVAL, "grad is NULL");
  if (!a->seeded) return fail(c, LBF_ESTATE, "lbf_adjoint_seed has not been called");
  ADJCHK(adj_reduce(a, adj_part(a), lbf::NPAR, a->lay.nblocks, adj_acc(a)));
  HIPCHK(c, hipMemcpyAsync(grad, adj_acc(a), lbf::NPAR * sizeof(double), hipMemcpyDeviceToHost, a->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipStreamSynchronize(a->stream), "hipStreamSynchronize");
  if (!all_finite(grad, lbf::NPAR))
    return fail(c, LBF_ENAN, "non-finite gradient: the reverse sweep overflowed");
  return LBF_OK;
}

lbf_status lbf_adjoint_state(lbf_adj* a, double* pops, double* aux) {
  if (!a) return LBF_EINVAL;
  lbf_ctx* c = a->c;
  if (!pops || !aux) return fail(c, LBF_EINVAL, "output is NULL");
  if (!a->seeded) return fail(c, LBF_ESTATE, "lbf_adjoint_seed has not been called");
  ADJCHK(read_back(c, adj_lp(a, a->cur), (long long)c->nlat * c->Q, pops));
  ADJCHK(read_back(c, adj_la(a, a->cur), c->naux, aux));
  // add each cell's population scalars (g_p: plane naux + p, h: naux + N)
  const long long nc = c->ncell;
  double* sc = new (std::nothrow) double[(size_t)(c->N + 1) * nc];
  if (!sc) return fail(c, LBF_ENOMEM, "host scratch");
  const size_t elt = c->lay.elt;
  const lbf_status s = read_back(c, static_cast<char*>(adj_la(a, a->cur)) + (size_t)c->naux * nc * elt,
                                 c->N + 1, sc);
  if (s == LBF_OK)
    for (int l = 1; l <= c->N + 1; ++l)
      for (int i = 0; i < c->Q; ++i) {
        double* dst = pops + ((long long)l * c->Q + i) * nc;
        const double* add = sc + (long long)(l - 1) * nc;
        for (long long k = 0; k < nc; ++k) dst[k] += add[k];
      }
  delete[] sc;
  return s;
}

lbf_status lbf_adjoint_destroy(lbf_adj* a) {
  delete a;
  return LBF_OK;
}

}  // extern "C"

// ----- batched cases ---------------------------------------------------
namespace {

// Blocks of each pass of group g with row tile variant v (the geometry the
// case table gets: about 4096 collide blocks over the group, split by cell
// counts; moment blocks of MOMENT_THREADS cells).
void batch_blocks(const std::vector<lbf_ctx*>& ctx, int v, long long& cblocks, long long& mblocks) {
  long long total = 0;
  for (lbf_ctx* c : ctx) total += c->ncell;
  cblocks = mblocks = 0;
  for (lbf_ctx* c : ctx) {
    int ntx, chunk, nb;
    lbf::batch_geometry(c->kp, lbf::BATCH_TILES[v], (4096LL * c->ncell + total - 1) / total, ntx, chunk, nb);
    cblocks += nb;
    mblocks += (c->ncell + lbf::MOMENT_THREADS - 1) / lbf::MOMENT_THREADS;
  }
}

// Device bytes of a group's table: the cases, then the moment pass's
// block-to-case map, then the collide pass's (sized for the tile variant
// with the most blocks).
size_t batch_table_bytes(const std::vector<lbf_ctx*>& ctx) {
  long long cmax = 0, mb = 0;
  for (int v = 0; v < 3; ++v) {
    long long cb, m;
    batch_blocks(ctx, v, cb, m);
    cmax = cb > cmax ? cb : cmax;
    mb = m;
  }
  return lbf::align256(ctx.size() * sizeof(lbf::BatchCase<float>) + (size_t)(mb + cmax) * sizeof(int));
}

lbf_status batch_validate(lbf_ctx* const* ctxs, int n, std::string& err) {
  if (!ctxs || n < 1) {
    err = "no contexts";
    return LBF_EINVAL;
  }
  for (int k = 0; k < n; ++k) {
    lbf_ctx* c = ctxs[k];
    if (!c) {
      err = "NULL context";
      return LBF_EINVAL;
    }
    if (!c->ops->batch) {
      err = "batched steps are built for 2D";
      return LBF_ENOTSUP;
    }
    if (c->prm.precision != ctxs[0]->prm.precision || c->device != ctxs[0]->device) {
      err = "contexts of a batch share the precision and the device";
      return LBF_EINVAL;
    }
    if (!c->initialized) {
      err = "lbf_init_fields has not been called on every context";
      return LBF_ESTATE;
    }
    for (int j = 0; j < k; ++j)
      if (ctxs[j] == c) {
        err = "a context appears twice";
        return LBF_EINVAL;
      }
  }
  return LBF_OK;
}

// Case table of group g for row tile variant v: geometry per case (about
// 4096 collide blocks over the group, split by cell counts), block offsets.
template <typename S>
void batch_table(const lbf_batch_group& g, int v, const char* own_base, std::vector<lbf::BatchCase<S>>& t,
                 std::vector<int>& map, int& cblocks, int& mblocks) {
  long long total = 0;
  for (lbf_ctx* c : g.ctx) total += c->ncell;
  t.resize(g.ctx.size());
  cblocks = mblocks = 0;
  for (size_t k = 0; k < g.ctx.size(); ++k) {
    lbf_ctx* c = g.ctx[k];
    lbf::BatchCase<S>& b = t[k];
    b.P = kp_ptr(c);
    b.soff = g.soff[k];
    b.pop_bytes = (long long)c->lay.pop_bytes;
    for (int j = 0; j < 2; ++j) {
      b.pop_off[j] = static_cast<const char*>(pop_ptr(c, j)) - own_base;
      b.aux_off[j] = static_cast<const char*>(aux_ptr(c, j)) - own_base;
    }
    b.cur = g.cur0[k];
    const long long target = (4096LL * c->ncell + total - 1) / total;
    lbf::batch_geometry(c->kp, lbf::BATCH_TILES[v], target, b.ntx, b.chunk, b.nblocks);
    b.nty = 1;
    b.mblocks = (int)((c->ncell + lbf::MOMENT_THREADS - 1) / lbf::MOMENT_THREADS);
    b.first_cblock = cblocks;
    b.first_mblock = mblocks;
    cblocks += b.nblocks;
    mblocks += b.mblocks;
  }
  // block-to-case maps after the table: moment blocks, then collide blocks
  static_assert(sizeof(lbf::BatchCase<S>) % sizeof(int) == 0, "maps follow the table in ints");
  const int map0 = (int)(t.size() * sizeof(t[0]) / sizeof(int));
  map.assign((size_t)mblocks + cblocks, 0);
  for (size_t k = 0; k < t.size(); ++k) {
    t[k].map_m = map0;
    t[k].map_c = map0 + mblocks;
    for (int j = 0; j < t[k].mblocks; ++j) map[t[k].first_mblock + j] = (int)k;
    for (int j = 0; j < t[k].nblocks; ++j) map[mblocks + t[k].first_cblock + j] = (int)k;
  }
}

// A captured graph holds the launches of the case tables it was captured
// with (tile variant, block counts); rewriting a table makes it stale, so it
// is dropped and lbf_batch_replay refuses until the next lbf_batch_capture.
void batch_drop_graph(lbf_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

lbf_status batch_set_variant(lbf_batch* b, int gi, int v) {
  lbf_batch_group& g = b->g[gi];
  lbf_ctx* c0 = b->first;
  void* dst = b->base + g.off;
  batch_drop_graph(b);
  std::vector<int> map;
  std::vector<char> img;
  int cblocks = 0, mblocks = 0;
  auto pack = [&](const auto& t) {
    const size_t tb = t.size() * sizeof(t[0]);
    img.resize(tb + map.size() * sizeof(int));
    memcpy(img.data(), t.data(), tb);
    memcpy(img.data() + tb, map.data(), map.size() * sizeof(int));
  };
  if (c0->prm.precision == LBF_FP64) {
    std::vector<lbf::BatchCase<double>> t;
    batch_table<double>(g, v, b->own_base, t, map, cblocks, mblocks);
    pack(t);
  } else {
    std::vector<lbf::BatchCase<float>> t;
    batch_table<float>(g, v, b->own_base, t, map, cblocks, mblocks);
    pack(t);
  }
  if (img.size() > batch_table_bytes(g.ctx))  // the sizing and the table must agree on the geometry
    return fail(c0, LBF_EINVAL, "batch case table larger than its reserved space");
  HIPCHK(c0, hipMemcpyAsync(dst, img.data(), img.size(), hipMemcpyHostToDevice, b->stream), "hipMemcpyAsync");
  HIPCHK(c0, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  g.cblocks = cblocks;
  g.mblocks = mblocks;
  g.variant = v;
  return LBF_OK;
}

// One batched step of every group at the given parity (the state buffers
// read are cur0 ^ parity, at their table offsets from own_base), or from
// packed batch state src to dst.  With
// LBF_BATCH_CONCURRENT the groups after the first run on side streams forked
// from and joined back to the batch's stream (parallel branches when
// captured).
lbf_status batch_launch(lbf_batch* b, int parity, const void* src = nullptr, void* dst = nullptr) {
  lbf_ctx* c0 = b->first;
  const bool packed = src && dst;
  if (!packed) src = dst = b->own_base;
  const int pers = (b->launch & LBF_BATCH_PERSISTENT) ? (b->grid > 0 ? b->grid : -1) : 0;
  int ngroup = 0;
  for (int gi = 0; gi < lbf::MAXP; ++gi) ngroup += !b->g[gi].ctx.empty();
  const bool conc = (b->launch & LBF_BATCH_CONCURRENT) && ngroup > 1;
  if (conc) HIPCHK(c0, hipEventRecord(b->fork, b->stream), "hipEventRecord");
  bool first = true;
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    lbf_batch_group& g = b->g[gi];
    if (g.ctx.empty()) continue;
    const lbf::Ops* ops = g.ctx[0]->ops;
    const int n = (int)g.ctx.size();
    const bool side = conc && !first;
    hipStream_t s = side ? b->side[gi] : b->stream;
    first = false;
    if (side) HIPCHK(c0, hipStreamWaitEvent(s, b->fork, 0), "hipStreamWaitEvent");
    HIPCHK(c0, ops->batch(0, g.variant, b->base + g.off, n, g.mblocks, parity, src, dst, packed, pers, s),
           "batched moments");
    HIPCHK(c0, ops->batch(1, g.variant, b->base + g.off, n, g.cblocks, parity, src, dst, packed, pers, s),
           "batched collide");
    if (side) {
      HIPCHK(c0, hipEventRecord(b->join[gi], s), "hipEventRecord");
      HIPCHK(c0, hipStreamWaitEvent(b->stream, b->join[gi], 0), "hipStreamWaitEvent");
    }
  }
  return LBF_OK;
}

void batch_release_streams(lbf_batch* b) {
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    if (b->side[gi]) (void)hipStreamDestroy(b->side[gi]);
    if (b->join[gi]) (void)hipEventDestroy(b->join[gi]);
    b->side[gi] = nullptr;
    b->join[gi] = nullptr;
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  b->fork = nullptr;
}

lbf_status batch_check_members(lbf_batch* b) {
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    lbf_batch_group& g = b->g[gi];
    for (size_t k = 0; k < g.ctx.size(); ++k)
      if (g.ctx[k]->cur != (g.cur0[k] ^ b->parity))
        return fail(b->first, LBF_ESTATE, "a member context was stepped outside the batch");
  }
  return LBF_OK;
}

void batch_advance(lbf_batch* b, int nsteps) {
  b->parity ^= (nsteps & 1);
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    lbf_batch_group& g = b->g[gi];
    for (size_t k = 0; k < g.ctx.size(); ++k) {
      g.ctx[k]->cur = g.cur0[k] ^ b->parity;
      g.ctx[k]->steps += nsteps;
    }
  }
}

}  // namespace

extern "C" {

lbf_status lbf_batch_bytes(lbf_ctx* const* ctxs, int n, size_t* bytes) {
  if (!bytes) return LBF_EINVAL;
  std::string err;
  const lbf_status st = batch_validate(ctxs, n, err);
  if (st != LBF_OK) return st;
  std::vector<lbf_ctx*> grp[lbf::MAXP];
  for (int k = 0; k < n; ++k) grp[ctxs[k]->N - 1].push_back(ctxs[k]);
  size_t o = 0;
  for (int gi = 0; gi < lbf::MAXP; ++gi)
    if (!grp[gi].empty()) o += batch_table_bytes(grp[gi]);
  *bytes = o;
  return LBF_OK;
}

lbf_status lbf_batch_create(lbf_ctx* const* ctxs, int n, void* dev_buf, size_t bytes, void* hip_stream,
                            lbf_batch** out) {
  if (!out) return LBF_EINVAL;
  *out = nullptr;
  std::string err;
  const lbf_status st = batch_validate(ctxs, n, err);
  if (st != LBF_OK) {
    if (ctxs && n > 0 && ctxs[0]) fail(ctxs[0], st, err);
    return st;
  }
  size_t need;
  lbf_batch_bytes(ctxs, n, &need);
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) & 255) || bytes < need)
    return fail(ctxs[0], LBF_EINVAL, "batch buffer missing, unaligned or smaller than lbf_batch_bytes");
  if (!hip_stream) return fail(ctxs[0], LBF_EINVAL, "a batch needs a non-default stream (graph capture)");
  lbf_batch* b = new (std::nothrow) lbf_batch();
  if (!b) return LBF_ENOMEM;
  b->first = ctxs[0];
  b->ncase = n;
  b->base = static_cast<char*>(dev_buf);
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->parity = 0;
  b->graph = nullptr;
  b->exec = nullptr;
  b->graph_parity = 0;
  b->own_base = nullptr;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < 2; ++j)
      for (char* p : {static_cast<char*>(pop_ptr(ctxs[k], j)), static_cast<char*>(aux_ptr(ctxs[k], j))})
        if (!b->own_base || p < b->own_base) b->own_base = p;
  b->launch = 0;
  b->grid = 0;
  b->fork = nullptr;
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    b->side[gi] = nullptr;
    b->join[gi] = nullptr;
  }
  size_t so = 0;
  for (int k = 0; k < n; ++k) {
    lbf_batch_group& g = b->g[ctxs[k]->N - 1];
    g.ctx.push_back(ctxs[k]);
    g.cur0.push_back(ctxs[k]->cur);
    g.user.push_back(k);
    g.soff.push_back((long long)so);
    so += lbf::align256(ctxs[k]->lay.pop_bytes + ctxs[k]->lay.aux_bytes);
  }
  b->state_bytes = so;
  size_t o = 0;
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    lbf_batch_group& g = b->g[gi];
    if (g.ctx.empty()) continue;
    g.off = o;
    o += batch_table_bytes(g.ctx);
    const lbf_status s2 = batch_set_variant(b, gi, 1);
    if (s2 != LBF_OK) {
      delete b;
      return s2;
    }
  }
  // the phase-count groups on parallel streams when there is more than one
  // (measured faster than one stream, and bitwise the same)
  int ngroup = 0;
  for (int gi = 0; gi < lbf::MAXP; ++gi) ngroup += !b->g[gi].ctx.empty();
  if (ngroup > 1) {
    const lbf_status s3 = lbf_batch_set_launch(b, LBF_BATCH_CONCURRENT, 0);
    if (s3 != LBF_OK) {
      lbf_batch_destroy(b);
      return s3;
    }
  }
  *out = b;
  return LBF_OK;
}

lbf_status lbf_batch_set_tiles(lbf_batch* b, const int* tile) {
  if (!b || !tile) return LBF_EINVAL;
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    if (b->g[gi].ctx.empty() || tile[gi] == 0) continue;
    int v = -1;
    for (int k = 0; k < 3; ++k)
      if (lbf::BATCH_TILES[k] == tile[gi]) v = k;
    if (v < 0) return fail(b->first, LBF_EINVAL, "row tile must be 64, 128 or 256");
    ADJCHK(batch_set_variant(b, gi, v));
  }
  return LBF_OK;
}

lbf_status lbf_batch_set_launch(lbf_batch* b, unsigned flags, int grid) {
  if (!b) return LBF_EINVAL;
  lbf_ctx* c0 = b->first;
  if (flags & ~(LBF_BATCH_PERSISTENT | LBF_BATCH_CONCURRENT)) return fail(c0, LBF_EINVAL, "unknown launch flags");
  if (grid < 0 || grid % 8) return fail(c0, LBF_EINVAL, "grid must be 0 or a positive multiple of 8");
  if ((flags & LBF_BATCH_CONCURRENT) && !b->fork) {
    int prev = 0;
    HIPCHK(c0, hipGetDevice(&prev), "hipGetDevice");
    HIPCHK(c0, hipSetDevice(c0->device), "hipSetDevice");
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int gi = 0; gi < lbf::MAXP && e == hipSuccess; ++gi) {
      if (b->g[gi].ctx.empty()) continue;
      e = hipStreamCreateWithFlags(&b->side[gi], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[gi], hipEventDisableTiming);
    }
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
      batch_release_streams(b);
      return hip_fail(c0, e, "side streams of a concurrent batch");
    }
  }
  if ((flags & LBF_BATCH_PERSISTENT) && grid == 0) {
    // Query the resident block counts of every pass, tile and state form now
    // (no launch), not during a later graph capture.
    char one = 0;
    for (int gi = 0; gi < lbf::MAXP; ++gi) {
      const lbf_batch_group& g = b->g[gi];
      if (g.ctx.empty()) continue;
      const lbf::Ops* ops = g.ctx[0]->ops;
      for (int v = 0; v < 3; ++v)
        for (int pass = 0; pass < 2; ++pass) {
          for (int packed = 0; packed < 2; ++packed)
            HIPCHK(c0, ops->batch(pass, v, b->base + g.off, (int)g.ctx.size(), 0, 0, &one, &one, packed != 0, -1,
                                  b->stream),
                   "occupancy query");
        }
    }
  }
  batch_drop_graph(b);
  b->launch = flags;
  b->grid = grid;
  return LBF_OK;
}

lbf_status lbf_batch_tune(lbf_batch* b, int trial_steps, int* tile) {
  if (!b) return LBF_EINVAL;
  if (trial_steps < 1) return fail(b->first, LBF_EINVAL, "trial_steps must be >= 1");
  lbf_ctx* c0 = b->first;
  ADJCHK(batch_check_members(b));
  hipEvent_t e0, e1;
  HIPCHK(c0, hipEventCreate(&e0), "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c0, LBF_EDEVICE, "hipEventCreate");
  }
  lbf_status result = LBF_OK;
  const int pers = (b->launch & LBF_BATCH_PERSISTENT) ? (b->grid > 0 ? b->grid : -1) : 0;
  for (int gi = 0; gi < lbf::MAXP && result == LBF_OK; ++gi) {
    lbf_batch_group& g = b->g[gi];
    if (tile) tile[gi] = 0;
    if (g.ctx.empty()) continue;
    const lbf::Ops* ops = g.ctx[0]->ops;
    const int n = (int)g.ctx.size();
    float best = 0.f;
    int bestv = 1;
    for (int v = 0; v < 3 && result == LBF_OK; ++v) {
      result = batch_set_variant(b, gi, v);
      if (result != LBF_OK) break;
      // Trial passes read the current state and write only the scratch
      // buffers (the parity is not advanced): the state is unchanged.
      float ms = 0.f;
      hipError_t e = hipSuccess;
      for (int rep = 0; rep <= trial_steps && e == hipSuccess; ++rep) {
        if (rep == 1) e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess)
          e = ops->batch(0, v, b->base + g.off, n, g.mblocks, b->parity, b->own_base, b->own_base, false, pers,
                         b->stream);
        if (e == hipSuccess)
          e = ops->batch(1, v, b->base + g.off, n, g.cblocks, b->parity, b->own_base, b->own_base, false, pers,
                         b->stream);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        result = hip_fail(c0, e, "batch autotune");
        break;
      }
      if (v == 0 || ms < best) {
        best = ms;
        bestv = v;
      }
    }
    if (result == LBF_OK) result = batch_set_variant(b, gi, bestv);
    if (tile) tile[gi] = lbf::BATCH_TILES[bestv];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return result;
}

lbf_status lbf_batch_step(lbf_batch* b, int nsteps) {
  if (!b) return LBF_EINVAL;
  if (nsteps < 0) return fail(b->first, LBF_EINVAL, "nsteps must be >= 0");
  ADJCHK(batch_check_members(b));
  for (int s = 0; s < nsteps; ++s) {
    ADJCHK(batch_launch(b, b->parity));
    batch_advance(b, 1);
  }
  return LBF_OK;
}

lbf_status lbf_batch_capture(lbf_batch* b) {
  if (!b) return LBF_EINVAL;
  lbf_ctx* c0 = b->first;
  ADJCHK(batch_check_members(b));
  batch_drop_graph(b);
  HIPCHK(c0, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  lbf_status st = batch_launch(b, b->parity);
  if (st == LBF_OK) st = batch_launch(b, b->parity ^ 1);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &graph);
  if (st != LBF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  HIPCHK(c0, e, "hipStreamEndCapture");
  b->graph = graph;
  HIPCHK(c0, hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  b->graph_parity = b->parity;
  return LBF_OK;
}

lbf_status lbf_batch_replay(lbf_batch* b, int times) {
  if (!b) return LBF_EINVAL;
  lbf_ctx* c0 = b->first;
  if (!b->exec) return fail(c0, LBF_ESTATE, "lbf_batch_capture has not been called");
  if (times < 0) return fail(c0, LBF_EINVAL, "times must be >= 0");
  if (b->parity != b->graph_parity)
    return fail(c0, LBF_ESTATE, "an odd number of eager batch steps since the capture");
  ADJCHK(batch_check_members(b));
  for (int k = 0; k < times; ++k) HIPCHK(c0, hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
  batch_advance(b, 2 * times);
  return LBF_OK;
}

lbf_status lbf_batch_destroy(lbf_batch* b) {
  if (!b) return LBF_OK;
  batch_drop_graph(b);
  batch_release_streams(b);
  delete b;
  return LBF_OK;
}

lbf_status lbf_batch_state_bytes(const lbf_batch* b, size_t* bytes) {
  if (!b || !bytes) return LBF_EINVAL;
  *bytes = b->state_bytes;
  return LBF_OK;
}

lbf_status lbf_batch_state_to_device(lbf_batch* b, void* dst) {
  if (!b) return LBF_EINVAL;
  lbf_ctx* c0 = b->first;
  if (!dst || (reinterpret_cast<uintptr_t>(dst) & 255))
    return fail(c0, LBF_EINVAL, "dst must be a 256-byte aligned device buffer");
  ADJCHK(batch_check_members(b));
  char* d = static_cast<char*>(dst);
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    lbf_batch_group& g = b->g[gi];
    for (size_t k = 0; k < g.ctx.size(); ++k) {
      lbf_ctx* c = g.ctx[k];
      const int cur = g.cur0[k] ^ b->parity;
      HIPCHK(c0, hipMemcpyAsync(d + g.soff[k], pop_ptr(c, cur), c->lay.pop_bytes, hipMemcpyDeviceToDevice, b->stream),
             "hipMemcpyAsync");
      HIPCHK(c0, hipMemcpyAsync(d + g.soff[k] + c->lay.pop_bytes, aux_ptr(c, cur), c->lay.aux_bytes,
                                hipMemcpyDeviceToDevice, b->stream),
             "hipMemcpyAsync");
    }
  }
  return LBF_OK;
}

lbf_status lbf_batch_state_from_device(lbf_batch* b, const void* src, long long advance) {
  if (!b) return LBF_EINVAL;
  lbf_ctx* c0 = b->first;
  if (!src || (reinterpret_cast<uintptr_t>(src) & 255))
    return fail(c0, LBF_EINVAL, "src must be a 256-byte aligned device buffer");
  if (advance < 0) return fail(c0, LBF_EINVAL, "advance must be >= 0");
  ADJCHK(batch_check_members(b));
  const char* s = static_cast<const char*>(src);
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    lbf_batch_group& g = b->g[gi];
    for (size_t k = 0; k < g.ctx.size(); ++k) {
      lbf_ctx* c = g.ctx[k];
      const int cur = g.cur0[k] ^ b->parity;
      HIPCHK(c0, hipMemcpyAsync(pop_ptr(c, cur), s + g.soff[k], c->lay.pop_bytes, hipMemcpyDeviceToDevice, b->stream),
             "hipMemcpyAsync");
      HIPCHK(c0, hipMemcpyAsync(aux_ptr(c, cur), s + g.soff[k] + c->lay.pop_bytes, c->lay.aux_bytes,
                                hipMemcpyDeviceToDevice, b->stream),
             "hipMemcpyAsync");
      c->steps += advance;
      c->nan_flag = false;
    }
  }
  return LBF_OK;
}

lbf_status lbf_batch_step_states(lbf_batch* b, const void* src, void* dst) {
  if (!b) return LBF_EINVAL;
  lbf_ctx* c0 = b->first;
  if (!src || !dst || src == dst) return fail(c0, LBF_EINVAL, "src and dst must be distinct packed batch states");
  if ((reinterpret_cast<uintptr_t>(src) & 255) || (reinterpret_cast<uintptr_t>(dst) & 255))
    return fail(c0, LBF_EINVAL, "packed batch states must be 256-byte aligned");
  return batch_launch(b, 0, src, dst);
}

}  // extern "C"

// ----- batched reverse step ---------------------------------------------
// Every case keeps a single-case adjoint context (its own adjoint buffer, on
// the batch's stream); the per-step passes run as one launch per phase
// count over the case tables, the seed, the start term and the gradient
// reduction (once per sweep) case by case.
struct lbf_batch_adj {
  lbf_batch* b;
  char* base;
  std::vector<lbf_adj*> adj;  // caller order
  struct Group {
    size_t off;  // case table offset in the device buffer
    int n, cblocks, tblocks, ctblocks;  // blocks of the per-cell collide reverse, the gather, the tiled collide reverse
  } g[lbf::MAXP];
  int cur;
  bool seeded;
};

namespace {

// case table, then the cases' parameter blocks
size_t batch_adj_table_bytes(int n) {
  return lbf::batch_adj_params_offset(n) + lbf::align256((size_t)n * sizeof(lbf::KParams));
}

// Buffer layout: per group a case table, then each case's adjoint buffer in
// caller order.  Returns the total; fills the offsets if given.
size_t batch_adj_layout(const lbf_batch* b, size_t* table_off, std::vector<size_t>* case_off) {
  size_t o = 0;
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    if (table_off) table_off[gi] = o;
    if (!b->g[gi].ctx.empty()) o += batch_adj_table_bytes((int)b->g[gi].ctx.size());
  }
  std::vector<const lbf_ctx*> byuser(b->ncase, nullptr);
  for (int gi = 0; gi < lbf::MAXP; ++gi)
    for (size_t k = 0; k < b->g[gi].ctx.size(); ++k) byuser[b->g[gi].user[k]] = b->g[gi].ctx[k];
  if (case_off) case_off->assign(b->ncase, 0);
  for (int u = 0; u < b->ncase; ++u) {
    if (case_off) (*case_off)[u] = o;
    o += lbf::align256(lbf::make_adj_layout(&byuser[u]->prm, byuser[u]->lay).total);
  }
  return o;
}

void batch_adj_free(lbf_batch_adj* ba) {
  for (lbf_adj* a : ba->adj) delete a;
  delete ba;
}

}  // namespace

extern "C" {

lbf_status lbf_batch_adjoint_bytes(const lbf_batch* b, size_t* bytes) {
  if (!b || !bytes) return LBF_EINVAL;
  for (int gi = 0; gi < lbf::MAXP; ++gi)
    for (lbf_ctx* c : b->g[gi].ctx) {
      if (!c->ops->batch_adjoint) return LBF_ENOTSUP;
      size_t one = 0;
      const lbf_status st = lbf_adjoint_bytes(&c->prm, &one);  // the single-case limits hold per case
      if (st != LBF_OK) return st;
    }
  *bytes = batch_adj_layout(b, nullptr, nullptr);
  return LBF_OK;
}

lbf_status lbf_batch_adjoint_create(lbf_batch* b, void* dev_buf, size_t bytes, lbf_batch_adj** out) {
  if (!b || !out) return LBF_EINVAL;
  *out = nullptr;
  lbf_ctx* c0 = b->first;
  size_t need = 0;
  if (lbf_batch_adjoint_bytes(b, &need) != LBF_OK)
    return fail(c0, LBF_ENOTSUP, "the batched reverse step is built for 2D float32 and float64");
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) & 255) || bytes < need)
    return fail(c0, LBF_EINVAL, "batched adjoint buffer missing, unaligned or smaller than lbf_batch_adjoint_bytes");
  lbf_batch_adj* ba = new (std::nothrow) lbf_batch_adj();
  if (!ba) return LBF_ENOMEM;
  ba->b = b;
  ba->base = static_cast<char*>(dev_buf);
  ba->cur = 0;
  ba->seeded = false;
  size_t toff[lbf::MAXP];
  std::vector<size_t> coff;
  batch_adj_layout(b, toff, &coff);
  ba->adj.assign(b->ncase, nullptr);
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    lbf_batch_group& g = b->g[gi];
    lbf_batch_adj::Group& G = ba->g[gi];
    G.off = toff[gi];
    G.n = (int)g.ctx.size();
    G.cblocks = G.tblocks = G.ctblocks = 0;
    if (g.ctx.empty()) continue;
    std::vector<lbf::BatchAdjCase> t(g.ctx.size());
    std::vector<lbf::KParams> kps(g.ctx.size());
    for (size_t k = 0; k < g.ctx.size(); ++k) {
      lbf_ctx* c = g.ctx[k];
      lbf_adj* a = new (std::nothrow) lbf_adj();
      if (!a) {
        batch_adj_free(ba);
        return LBF_ENOMEM;
      }
      a->c = c;
      a->lay = lbf::make_adj_layout(&c->prm, c->lay);
      a->base = ba->base + coff[g.user[k]];
      a->stream = b->stream;
      a->cur = 0;
      a->seeded = false;
      a->J = 0.0;
      ba->adj[g.user[k]] = a;
      lbf::BatchAdjCase& bc = t[k];
      kps[k] = c->kp;
      bc.soff = g.soff[k];
      bc.pop_bytes = (long long)c->lay.pop_bytes;
      for (int j = 0; j < 2; ++j) {
        bc.lp_off[j] = static_cast<char*>(adj_lp(a, j)) - ba->base;
        bc.la_off[j] = static_cast<char*>(adj_la(a, j)) - ba->base;
      }
      bc.work_off = static_cast<char*>(adj_work(a)) - ba->base;
      bc.part_off = reinterpret_cast<char*>(adj_part(a)) - ba->base;
      // the single-case tile geometry, which the gradient rows follow
      const lbf::Geometry geo = c->prm.precision == LBF_FP64
                                    ? lbf::step_geometry<lbf::CfgOf<2, 1, double, double>>(c->kp)
                                    : lbf::step_geometry<lbf::CfgOf<2, 1, float, float>>(c->kp);
      bc.ntx = geo.ntx;
      bc.nty = geo.nty;
      bc.chunk = geo.chunk;
      bc.nblocks = geo.nblocks;
      bc.first_tblock = G.tblocks;
      G.tblocks += bc.nblocks;
      // the single-case form of the collide reverse: one thread per cell
      // (256-cell blocks) or the tiles of the step geometry
      const bool tiled = lbf::collide_reverse_tiled(c->N, geo.nblocks);
      bc.cblocks = tiled ? 0 : a->lay.cblocks;
      bc.first_cblock = G.cblocks;
      G.cblocks += bc.cblocks;
      bc.ctblocks = tiled ? geo.nblocks : 0;
      bc.first_ctblock = G.ctblocks;
      G.ctblocks += bc.ctblocks;
    }
    hipError_t e = hipMemcpyAsync(ba->base + G.off, t.data(), t.size() * sizeof(t[0]), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ba->base + G.off + lbf::batch_adj_params_offset(G.n), kps.data(),
                         kps.size() * sizeof(kps[0]), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
      batch_adj_free(ba);
      return hip_fail(c0, e, "batched adjoint case table");
    }
  }
  *out = ba;
  return LBF_OK;
}

lbf_status lbf_batch_adjoint_seed(lbf_batch_adj* ba, int objective, const void* state, double* J) {
  if (!ba) return LBF_EINVAL;
  lbf_batch* b = ba->b;
  if (!state) return fail(b->first, LBF_EINVAL, "state is NULL");
  const char* st = static_cast<const char*>(state);
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    lbf_batch_group& g = b->g[gi];
    for (size_t k = 0; k < g.ctx.size(); ++k) {
      lbf_adj* a = ba->adj[g.user[k]];
      const char* pin = st + g.soff[k];
      double Jk = 0.0;
      const lbf_status s = adj_seed_at(a, objective, pin, pin + g.ctx[k]->lay.pop_bytes, &Jk);
      if (s != LBF_OK) {
        if (s != LBF_EDEVICE) fail(b->first, s, g.ctx[k]->err);
        return s;
      }
      if (J) J[g.user[k]] = Jk;
    }
  }
  ba->cur = 0;
  ba->seeded = true;
  return LBF_OK;
}

lbf_status lbf_batch_adjoint_step(lbf_batch_adj* ba, const void* state, const void* next) {
  if (!ba) return LBF_EINVAL;
  lbf_batch* b = ba->b;
  lbf_ctx* c0 = b->first;
  if (!ba->seeded) return fail(c0, LBF_ESTATE, "lbf_batch_adjoint_seed has not been called");
  if (!state || !next) return fail(c0, LBF_EINVAL, "state and next must be packed batch states");
  // the phase-count groups on parallel branches, as in batch_launch
  int ngroup = 0;
  for (int gi = 0; gi < lbf::MAXP; ++gi) ngroup += ba->g[gi].n > 0;
  const bool conc = (b->launch & LBF_BATCH_CONCURRENT) && ngroup > 1;
  if (conc) HIPCHK(c0, hipEventRecord(b->fork, b->stream), "hipEventRecord");
  bool first = true;
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    const lbf_batch_adj::Group& G = ba->g[gi];
    if (!G.n) continue;
    const lbf::Ops* ops = b->g[gi].ctx[0]->ops;
    const bool side = conc && !first;
    hipStream_t s = side ? b->side[gi] : b->stream;
    first = false;
    if (side) HIPCHK(c0, hipStreamWaitEvent(s, b->fork, 0), "hipStreamWaitEvent");
    if (G.cblocks)
      HIPCHK(c0, ops->batch_adjoint(0, ba->base + G.off, G.n, G.cblocks, state, next, ba->cur, ba->base, s),
             "batched collide reverse (per cell)");
    if (G.ctblocks)
      HIPCHK(c0, ops->batch_adjoint(2, ba->base + G.off, G.n, G.ctblocks, state, next, ba->cur, ba->base, s),
             "batched collide reverse (tiled)");
    HIPCHK(c0, ops->batch_adjoint(1, ba->base + G.off, G.n, G.tblocks, state, next, ba->cur, ba->base, s),
           "batched gather");
    if (side) {
      HIPCHK(c0, hipEventRecord(b->join[gi], s), "hipEventRecord");
      HIPCHK(c0, hipStreamWaitEvent(b->stream, b->join[gi], 0), "hipStreamWaitEvent");
    }
  }
  ba->cur ^= 1;
  for (lbf_adj* a : ba->adj) a->cur = ba->cur;
  return LBF_OK;
}

lbf_status lbf_batch_adjoint_finish(lbf_batch_adj* ba, const void* state0) {
  if (!ba) return LBF_EINVAL;
  lbf_batch* b = ba->b;
  if (!ba->seeded) return fail(b->first, LBF_ESTATE, "lbf_batch_adjoint_seed has not been called");
  if (!state0) return fail(b->first, LBF_EINVAL, "state0 is NULL");
  const char* st = static_cast<const char*>(state0);
  for (int gi = 0; gi < lbf::MAXP; ++gi) {
    lbf_batch_group& g = b->g[gi];
    for (size_t k = 0; k < g.ctx.size(); ++k) {
      lbf_adj* a = ba->adj[g.user[k]];
      const char* pin = st + g.soff[k];
      ADJCHK(adj_pass(a, 6, pin, pin + g.ctx[k]->lay.pop_bytes, adj_lp(a, a->cur), adj_la(a, a->cur), nullptr,
                      nullptr, 0.0, 0.0));
    }
  }
  return LBF_OK;
}

lbf_status lbf_batch_adjoint_gradient(lbf_batch_adj* ba, double* grad) {
  if (!ba) return LBF_EINVAL;
  lbf_batch* b = ba->b;
  lbf_ctx* c0 = b->first;
  if (!grad) return fail(c0, LBF_EINVAL, "grad is NULL");
  if (!ba->seeded) return fail(c0, LBF_ESTATE, "lbf_batch_adjoint_seed has not been called");
  for (int u = 0; u < b->ncase; ++u) {
    lbf_adj* a = ba->adj[u];
    ADJCHK(adj_reduce(a, adj_part(a), lbf::NPAR, a->lay.nblocks, adj_acc(a)));
    HIPCHK(c0, hipMemcpyAsync(grad + (size_t)u * lbf::NPAR, adj_acc(a), lbf::NPAR * sizeof(double),
                              hipMemcpyDeviceToHost, b->stream),
           "hipMemcpyAsync");
  }
  HIPCHK(c0, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  if (!all_finite(grad, (long long)b->ncase * lbf::NPAR))
    return fail(c0, LBF_ENAN, "non-finite gradient of some case: its reverse sweep overflowed");
  return LBF_OK;
}

lbf_status lbf_batch_adjoint_destroy(lbf_batch_adj* ba) {
  if (ba) batch_adj_free(ba);
  return LBF_OK;
}

lbf_status lbf_step_count(const lbf_ctx* c, long long* steps) {
  if (!c || !steps) return LBF_EINVAL;
  *steps = c->steps;
  return LBF_OK;
}

lbf_status lbf_destroy(lbf_ctx* c) {
  delete c;
  return LBF_OK;
}

const char* lbf_last_error(const lbf_ctx* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"

// ----- bandwidth probe (context for the roofline) -------------------------
namespace {

__global__ void __launch_bounds__(512) probe_copy4(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(512) probe_read4(const float4* __restrict__ src, float* __restrict__ sink,
                                                   long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  float acc = 0.f;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float4 v = src[i];
    acc += v.x + v.y + v.z + v.w;
  }
  // a store only for an impossible sum keeps the loads without writing
  if (acc == -1.5f) sink[0] = acc;
}

}  // namespace

extern "C" {

lbf_status lbf_bandwidth_probe(void* a, void* b, size_t bytes, void* hip_stream, int reps, double* copy_bytes_per_s,
                               double* read_bytes_per_s) {
  if (!a || !b || a == b || bytes < 4096 || reps < 1 || !copy_bytes_per_s || !read_bytes_per_s) return LBF_EINVAL;
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) return LBF_EINVAL;
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const long long n = (long long)((bytes - 16) / 16);  // the last 16 bytes of b are the read sink
  const float4* src = static_cast<const float4*>(a);
  float4* dst = static_cast<float4*>(b);
  float* sink = reinterpret_cast<float*>(static_cast<char*>(b) + (size_t)n * 16);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return LBF_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return LBF_EDEVICE;
  }
  const int grids[4] = {1024, 4096, 16384, 65536};
  const int blocks[2] = {256, 512};
  double best_copy = 0.0, best_read = 0.0;
  hipError_t e = hipSuccess;
  for (int gi = 0; gi < 4 && e == hipSuccess; ++gi)
    for (int bi = 0; bi < 2 && e == hipSuccess; ++bi)
      for (int kind = 0; kind < 2 && e == hipSuccess; ++kind) {
        const dim3 grid(grids[gi]), block(blocks[bi]);
        for (int r = 0; r <= reps && e == hipSuccess; ++r) {
          if (r == 1) e = hipEventRecord(e0, s);
          if (kind == 0)
            hipLaunchKernelGGL(probe_copy4, grid, block, 0, s, src, dst, n);
          else
            hipLaunchKernelGGL(probe_read4, grid, block, 0, s, src, sink, n);
          if (e == hipSuccess) e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms > 0.f) {
          const double rate = (kind == 0 ? 2.0 : 1.0) * 16.0 * (double)n * reps / (ms * 1e-3);
          if (kind == 0 && rate > best_copy) best_copy = rate;
          if (kind == 1 && rate > best_read) best_read = rate;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return LBF_EDEVICE;
  *copy_bytes_per_s = best_copy;
  *read_bytes_per_s = best_read;
  return LBF_OK;
}

const char* lbf_status_string(lbf_status s) {
  switch (s) {
    case LBF_OK: return "ok";
    case LBF_EINVAL: return "invalid argument";
    case LBF_ENOMEM: return "buffer too small";
    case LBF_EDEVICE: return "HIP runtime error";
    case LBF_ENOTSUP: return "not supported";
    case LBF_ENAN: return "non-finite state";
    case LBF_ESTATE: return "call out of order";
  }
  return "unknown status";
}

}  // extern "C"
