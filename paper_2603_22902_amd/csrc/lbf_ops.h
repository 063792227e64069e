// Type-erased entry points of the kernels for one (dim, N, precision).
// Each precision lives in its own translation unit (float64 is compiled
// without floating-point contraction); the C ABI picks a table at run time.
#pragma once

#include <hip/hip_runtime.h>

#include "lbf_lattice.h"

namespace lbf {

// P is the host copy of the parameter block (launch geometry), dP the
// device copy the kernels read.  step launches the moments pass if
// (passes & 1) and the collide pass if (passes & 2).
struct Ops {
  hipError_t (*step)(const void* pin, void* pout, const void* ain, void* aout, double* mout,
                     int mfield, const KParams& P, const KParams* dP, hipStream_t s, bool moments,
                     int passes);
  hipError_t (*init)(const KParams& P, const KParams* dP, const double* fields, int has_u,
                     int has_p, void* pop, void* aux, hipStream_t s);
  hipError_t (*diag)(const KParams& P, const KParams* dP, const void* pop, const void* aux,
                     double* part, double* out, hipStream_t s);
  hipError_t (*widen)(const void* in, double* out, long long n, hipStream_t s);
  // Passes of the reverse step (lbf_adjoint_kernels.h); NULL where the
  // adjoint is not built (3D, float32 storage with float64 arithmetic).
  hipError_t (*adjoint)(int pass, const void* pin, const void* ain, const void* lpin, const void* lain,
                        void* lpout, void* laout, const void* mom, void* work, const KParams& P,
                        const KParams* dP, double* part, double A, double B, hipStream_t s);
  // Batched passes over a case table (lbf_batch.h), 2D only (NULL in 3D):
  // pass 0 moments, 1 collide with row tile BATCH_TILES[variant]; with src
  // and dst (packed: packed batch states) from src to dst, else the cases'
  // own buffers at offsets from src = dst; grid: 0 one block per work item,
  // > 0 that many persistent blocks, < 0 the resident block count
  // (lbf_batch.h batch_grid).
  hipError_t (*batch)(int pass, int variant, const void* cases, int ncase, int nblocks, int parity,
                      const void* src, void* dst, bool packed, int grid, hipStream_t s);
  // Batched reverse-step passes (lbf_batch_adjoint.h): pass 0 per-cell
  // collide reverse, 2 tiled collide reverse, 1 tiled gather; NULL where the
  // adjoint is not built.
  hipError_t (*batch_adjoint)(int pass, const void* cases, int ncase, int nblocks, const void* state,
                              const void* next, int parity, void* abase, hipStream_t s);
};

// dim 2 or 3, nphase 1..4; NULL if not built.  f32: float32 storage and
// arithmetic; f64: float64 throughout; mix: float32 storage, float64
// arithmetic.
const Ops* ops_f32(int dim, int nphase);
const Ops* ops_f64(int dim, int nphase);
const Ops* ops_mix(int dim, int nphase);

}  // namespace lbf

// Instantiation of one precision's table (used by the kernel units); ADJ = 1
// also builds the reverse step for 2D.
#define LBF_DEFINE_OPS(NAME, ST, RT, ADJ)                                                            \
  namespace lbf {                                                                                \
  template <int DIM, int NP>                                                                     \
  struct OpsImpl_##NAME {                                                                        \
    static hipError_t step(const void* pin, void* pout, const void* ain, void* aout,             \
                           double* mout, int mfield, const KParams& P, const KParams* dP,        \
                           hipStream_t s, bool moments, int passes) {                            \
      StepArgs<ST> a;                                                                            \
      a.pin = static_cast<const ST*>(pin);                                                       \
      a.pout = static_cast<ST*>(pout);                                                           \
      a.ain = static_cast<const ST*>(ain);                                                       \
      a.aout = static_cast<ST*>(aout);                                                           \
      a.mout = mout;                                                                             \
      a.mfield = mfield;                                                                         \
      return launch_step<DIM, NP, ST, RT>(a, P, dP, s, moments, passes);                         \
    }                                                                                            \
    static hipError_t init(const KParams& P, const KParams* dP, const double* fields, int has_u, \
                           int has_p, void* pop, void* aux, hipStream_t s) {                     \
      return launch_init<DIM, NP, ST>(P, dP, fields, has_u, has_p, static_cast<ST*>(pop),        \
                                      static_cast<ST*>(aux), s);                                 \
    }                                                                                            \
    static hipError_t diag(const KParams& P, const KParams* dP, const void* pop, const void* aux, \
                           double* part, double* out, hipStream_t s) {                           \
      return launch_diag<DIM, NP, ST, RT>(P, dP, static_cast<const ST*>(pop),                    \
                                          static_cast<const ST*>(aux), part, out, s);            \
    }                                                                                            \
    static hipError_t widen(const void* in, double* out, long long n, hipStream_t s) {           \
      return launch_widen<ST>(static_cast<const ST*>(in), out, n, s);                            \
    }                                                                                            \
    static hipError_t adjoint(int pass, const void* pin, const void* ain, const void* lpin,     \
                              const void* lain, void* lpout, void* laout, const void* mom,       \
                              void* work,                                                        \
                              const KParams& P, const KParams* dP, double* part, double A,       \
                              double B, hipStream_t s) {                                         \
      if constexpr (ADJ && DIM == 2)                                                             \
        return launch_adjoint<DIM, NP, ST, RT>(                                                  \
            pass, static_cast<const ST*>(pin), static_cast<const ST*>(ain),                      \
            static_cast<const ST*>(lpin), static_cast<const ST*>(lain), static_cast<ST*>(lpout), \
            static_cast<ST*>(laout), static_cast<const ST*>(mom), work, P, dP, part, A, B, s);   \
      else                                                                                       \
        return hipErrorNotSupported;                                                             \
    }                                                                                            \
    static hipError_t batch(int pass, int variant, const void* cases, int ncase, int nblocks,    \
                            int parity, const void* src, void* dst, bool packed, int grid,       \
                            hipStream_t s) {                                                     \
      if constexpr (DIM == 2)                                                                    \
        return launch_batch<NP, ST, RT>(pass, variant, cases, ncase, nblocks, parity, src, dst,  \
                                        packed, grid, s);                                        \
      else                                                                                       \
        return hipErrorNotSupported;                                                             \
    }                                                                                            \
    static hipError_t batch_adjoint(int pass, const void* cases, int ncase, int nblocks,         \
                                    const void* state, const void* next, int parity,             \
                                    void* abase, hipStream_t s) {                                \
      if constexpr (ADJ && DIM == 2)                                                             \
        return launch_batch_adjoint<NP, ST, RT>(pass, cases, ncase, nblocks, state, next,        \
                                                parity, abase, s);                               \
      else                                                                                       \
        return hipErrorNotSupported;                                                             \
    }                                                                                            \
    static constexpr Ops ops = {&step, &init, &diag, &widen,                                     \
                                (ADJ && DIM == 2) ? &adjoint : nullptr,                          \
                                DIM == 2 ? &batch : nullptr,                                     \
                                (ADJ && DIM == 2) ? &batch_adjoint : nullptr};                   \
  };                                                                                             \
  const Ops* NAME(int dim, int nphase) {                                                         \
    static const Ops* table[2][4] = {                                                            \
        {&OpsImpl_##NAME<2, 1>::ops, &OpsImpl_##NAME<2, 2>::ops, &OpsImpl_##NAME<2, 3>::ops,     \
         &OpsImpl_##NAME<2, 4>::ops},                                                            \
        {&OpsImpl_##NAME<3, 1>::ops, &OpsImpl_##NAME<3, 2>::ops, &OpsImpl_##NAME<3, 3>::ops,     \
         &OpsImpl_##NAME<3, 4>::ops}};                                                           \
    if (dim < 2 || dim > 3 || nphase < 1 || nphase > 4) return nullptr;                          \
    return table[dim - 2][nphase - 1];                                                           \
  }                                                                                              \
  }
