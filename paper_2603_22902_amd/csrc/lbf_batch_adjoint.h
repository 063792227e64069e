// Batched reverse step: the two per-step passes of the reverse step (collide
// reverse, tiled gather) for many 2D cases of one phase count, one launch
// each.  A block finds its case in the case table (binary search over the
// cases' first block numbers) and runs the single-case phase functions with
// the case's parameter block, read through a restrict pointer into a
// contiguous array of the group's blocks (scalar loads, as in the
// single-case kernels).  Each case keeps the block decomposition (tiles, or
// 256-cell blocks for the per-cell collide reverse) and the gradient rows of
// its single-case reverse step, so its gradient is bitwise the one a
// single-case sweep gives.
#pragma once

#include <hip/hip_runtime.h>

#include "lbf_adjoint_kernels.h"
#include "lbf_batch.h"

namespace lbf {

// One case of a batched reverse step.  The states x^n and x^{n+1} of a step
// are packed batch states (soff, pop_bytes as in BatchCase); the adjoint
// buffers are the case's own (layout of the single-case reverse step), given
// as byte offsets from the batched adjoint buffer, whose address the
// kernels take as an argument (global, not generic: see BatchCase).
struct BatchAdjCase {
  long long soff, pop_bytes;
  long long lp_off[2], la_off[2], work_off;
  long long part_off;                 // gradient rows of the case
  int cblocks, first_cblock;          // one-thread-per-cell collide reverse (0 where the case takes the tiled one)
  int ntx, nty, chunk, nblocks;       // tile geometry of both passes (single-case step geometry)
  int first_tblock;                   // the tiled gather, every case
  int ctblocks, first_ctblock;        // tiled collide reverse (nblocks where the case takes it, else 0)
};

// Which block-number range a pass's blocks count in.
enum BatchAdjRange { ADJ_CELLS = 0, ADJ_TILES = 1, ADJ_COLLIDE_TILES = 2 };

// Last case k with first[k] <= b (uniform across the block).  A case with
// no blocks in the range shares its first block with the next case, so the
// search never lands on it.
__device__ inline int batch_adj_case(const BatchAdjCase* cs, int ncase, int b, int range) {
  int lo = 0, hi = ncase - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int f = range == ADJ_CELLS ? cs[mid].first_cblock
                  : range == ADJ_TILES ? cs[mid].first_tblock
                                       : cs[mid].first_ctblock;
    if (f <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Arguments of a case's reverse step through x^n = state (its moments from
// x^{n+1} = next); the adjoint of x^{n+1} is in buffers `parity`.
template <class C>
__device__ inline AdjArgs<C> batch_adj_args(const BatchAdjCase& bc, const char* state, const char* next,
                                            int parity, char* abase) {
  using S = typename C::S;
  AdjArgs<C> a;
  a.pin = reinterpret_cast<const S*>(state + bc.soff);
  a.ain = reinterpret_cast<const S*>(state + bc.soff + bc.pop_bytes);
  a.mom = reinterpret_cast<const S*>(next + bc.soff + bc.pop_bytes);
  a.lpin = reinterpret_cast<const S*>(abase + bc.lp_off[parity]);
  a.lain = reinterpret_cast<const S*>(abase + bc.la_off[parity]);
  a.lpout = reinterpret_cast<S*>(abase + bc.lp_off[1 - parity]);
  a.laout = reinterpret_cast<S*>(abase + bc.la_off[1 - parity]);
  a.work = reinterpret_cast<typename C::R*>(abase + bc.work_off);
  return a;
}

__device__ inline double* batch_adj_part(const BatchAdjCase& bc, char* abase) {
  return reinterpret_cast<double*>(abase + bc.part_off);
}

template <class C>
__global__ void __launch_bounds__(ADJ_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
    batch_adj_collide_cell_kernel(const BatchAdjCase* __restrict__ cs, const KParams* __restrict__ kpa, int ncase,
                                  const char* __restrict__ state, const char* __restrict__ next, int parity,
                                  char* __restrict__ abase) {
  const int k = __builtin_amdgcn_readfirstlane(batch_adj_case(cs, ncase, blockIdx.x, ADJ_CELLS));
  const BatchAdjCase& bc = cs[k];
  const KParams& P = kpa[k];
  const AdjArgs<C> a = batch_adj_args<C>(bc, state, next, parity, abase);
  double g[NPAR];
#pragma unroll
  for (int j = 0; j < NPAR; ++j) g[j] = 0.0;
  const int lb = blockIdx.x - bc.first_cblock;
  const int cell = lb * ADJ_THREADS + threadIdx.x;
  if (cell < P.ncell) adj_collide_cell<C>(a, P, cell, g);
  block_sum_to<NPAR, true>(g, batch_adj_part(bc, abase) + (long long)lb * NPAR);
}

template <class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2)))
    batch_adj_collide_kernel(const BatchAdjCase* __restrict__ cs, const KParams* __restrict__ kpa, int ncase,
                             int nblocks, const char* __restrict__ state, const char* __restrict__ next,
                             int parity, char* __restrict__ abase) {
  __shared__ Smem<C> sm;
  const int Lg = xcd_remap(blockIdx.x, nblocks);
  const int k = __builtin_amdgcn_readfirstlane(batch_adj_case(cs, ncase, Lg, ADJ_COLLIDE_TILES));
  const BatchAdjCase& bc = cs[k];
  const KParams& P = kpa[k];
  const AdjArgs<C> a = batch_adj_args<C>(bc, state, next, parity, abase);
  const StepArgs<typename C::S> sa = fill_args<C>(a, bc.ntx, bc.nty, bc.chunk, bc.nblocks);
  const int t = Lg - bc.first_ctblock;
  collide_tile_block<C>(a, sa, P, block_pos_local<C>(sa, P, t), sm, batch_adj_part(bc, abase) + (long long)t * NPAR);
}

template <class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(4)))
    batch_adj_gather_kernel(const BatchAdjCase* __restrict__ cs, const KParams* __restrict__ kpa, int ncase,
                            int nblocks, const char* __restrict__ state, const char* __restrict__ next,
                            int parity, char* __restrict__ abase) {
  __shared__ FdaRing<C> ring;
  const int Lg = xcd_remap(blockIdx.x, nblocks);
  const int k = __builtin_amdgcn_readfirstlane(batch_adj_case(cs, ncase, Lg, ADJ_TILES));
  const BatchAdjCase& bc = cs[k];
  const KParams& P = kpa[k];
  const AdjArgs<C> a = batch_adj_args<C>(bc, state, next, parity, abase);
  StepArgs<typename C::S> sa;
  sa.ntx = bc.ntx;
  sa.nty = bc.nty;
  sa.chunk = bc.chunk;
  sa.nblocks = bc.nblocks;
  const int t = Lg - bc.first_tblock;
  gather_tile_block<C>(a, P, block_pos_local<C>(sa, P, t), ring, batch_adj_part(bc, abase) + (long long)t * NPAR);
}

// pass 0: one-thread-per-cell collide reverse over the 256-cell blocks of
// the cases that take it (N <= 2), 2: tiled collide reverse over the tiles
// of the cases that take it, 1: tiled gather over every case's tiles
// (collide_reverse_tiled decides per case); nblocks in all.  cases: the
// case table followed, at the next 256-byte boundary, by the cases'
// parameter blocks in table order, which the kernels read through a
// restrict pointer (scalar loads, no LDS copy).  abase: the batched adjoint
// buffer the table's offsets count from.
inline size_t batch_adj_params_offset(int ncase) {
  return ((size_t)ncase * sizeof(BatchAdjCase) + 255) & ~size_t(255);
}

template <int NP, typename S, typename R>
inline hipError_t launch_batch_adjoint(int pass, const void* cases, int ncase, int nblocks, const void* state,
                                       const void* next, int parity, void* abase, hipStream_t s) {
  using C = CfgOf<2, NP, S, R>;
  const auto* cs = static_cast<const BatchAdjCase*>(cases);
  const auto* kpa =
      reinterpret_cast<const KParams*>(static_cast<const char*>(cases) + batch_adj_params_offset(ncase));
  const char* st = static_cast<const char*>(state);
  const char* nx = static_cast<const char*>(next);
  char* ab = static_cast<char*>(abase);
  if (!st || !nx || !ab || nblocks < 1) return hipErrorInvalidValue;
  if (pass == 0) {
    if constexpr (NP <= 2)
      hipLaunchKernelGGL((batch_adj_collide_cell_kernel<C>), dim3(nblocks), dim3(ADJ_THREADS), 0, s, cs, kpa,
                         ncase, st, nx, parity, ab);
    else
      return hipErrorInvalidValue;
  } else if (pass == 2) {
    if constexpr (NP >= 2)
      hipLaunchKernelGGL((batch_adj_collide_kernel<C>), dim3(nblocks), dim3(C::NT), 0, s, cs, kpa, ncase, nblocks,
                         st, nx, parity, ab);
    else
      return hipErrorInvalidValue;
  } else if (pass == 1)
    hipLaunchKernelGGL((batch_adj_gather_kernel<C>), dim3(nblocks), dim3(C::NT), 0, s, cs, kpa, ncase, nblocks, st,
                       nx, parity, ab);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace lbf
