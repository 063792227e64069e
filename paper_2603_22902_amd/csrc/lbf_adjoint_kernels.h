// HIP kernels of the reverse (adjoint) step and their launchers.
//
//   adj_moment_kernel        pass 1: forward moments of x^n
//   adj_collide_*kernel      pass 2: reverse of the collide pass (N >= 3: row
//                            tiles marching the wall-normal axis with an LDS
//                            ring; N <= 2: one thread per cell)
//   adj_gather_*kernel       pass 3: transpose of the finite differences and
//                            of the moments (tiled like the collide reverse;
//                            the seed pass, one thread per cell, starts from
//                            the objective)
//   adj_objective_kernel     sums A = sum f_s psi, B = sum psi of a state
//   adj_seed_kernel          adjoints of phi, f_s of the objective
//   adj_init_latent_kernel   dependence of the initial state on L_p
//
// (The block partials are summed into the gradient by a kernel of the API
// unit, which does not depend on the precision.)
// The per-cell kernels use 256-thread blocks; the tiled ones one 128-cell row
// of a tile per block.  Each thread's parameter-gradient contributions are
// summed in a fixed order (wave shuffles, then waves) and added to its
// block's row of a running accumulator (rows by block, or by tile for the
// tiled kernels); the rows are reduced once, in row order, when the gradient
// is read.  A reverse run is thus deterministic.
#pragma once

#include <hip/hip_runtime.h>

#include "lbf_adjoint.h"
#include "lbf_kernels.h"

namespace lbf {

constexpr int ADJ_THREADS = 256;

// Sum NV per-thread values over a block of NT threads into row[0..NV)
// (ACC: add to the row, which accumulates this block's terms over the
// reverse steps; else overwrite).  Fixed order: wave shuffles, then waves.
template <int NV, bool ACC, int NT = ADJ_THREADS>
__device__ inline void block_sum_to(const double* g, double* row) {
  __shared__ double red[NT / 64][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double v = g[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w][threadIdx.x];
    double* dst = row + threadIdx.x;
    *dst = ACC ? *dst + s : s;
  }
}

// The same into part[blockIdx.x][NV].
template <int NV, bool ACC>
__device__ inline void block_sum(const double* g, double* part) {
  block_sum_to<NV, ACC>(g, part + (long long)blockIdx.x * NV);
}

template <class C>
__global__ void __launch_bounds__(ADJ_THREADS)
    adj_moment_kernel(AdjArgs<C> a, const KParams* __restrict__ kp) {
  const KParams& P = *kp;
  const int cell = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (cell < P.ncell) adj_moment_cell<C>(a, P, cell);
}

template <class C, bool SEED>
__global__ void __launch_bounds__(ADJ_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
    adj_gather_kernel(AdjArgs<C> a, const KParams* __restrict__ kp, double* __restrict__ part) {
  const KParams& P = *kp;
  double g[NPAR];
#pragma unroll
  for (int k = 0; k < NPAR; ++k) g[k] = 0.0;
  const int cell = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (cell < P.ncell) adj_gather_cell<C>(a, P, cell, SEED, g);
  block_sum<NPAR, true>(g, part);
}

// The gather with the FD-adjoint planes of the tile and a one-cell halo
// staged in an LDS ring of three layers, the block marching along the
// wall-normal axis like the forward collide kernel (a non-seed pass).
template <class C>
struct FdaRing {
  static constexpr int NF = AdjLayout<C>::F_DIV - AdjLayout<C>::F_GPHI + 1;
  typename C::R v[3][NF][C::F];
};

template <class C>
struct FdaLds {
  const FdaRing<C>* ring;
  int fc, w;
  __host__ __device__ typename C::R operator()(int k, int, int dl0, int dl1, int dw) const {
    return ring->v[slot(w + dw)][k - AdjLayout<C>::F_GPHI][fc + dl0 + dl1 * C::LX];
  }
};

template <class C>
__host__ __device__ inline void fda_fill(const AdjArgs<C>& a, const KParams& P, FdaRing<C>& r, const BlockPos& bp,
                                         int f, int w) {
  using L = AdjLayout<C>;
  const int lx = f % C::LX, ly = f / C::LX;
  int lat = wrapf(bp.tx0 + lx - 1, P.nx);
  if (C::DIM == 3) lat += wrapf(bp.ty0 + ly - 1, P.ny) * P.nx;
  const int cell = w * (int)P.area + lat;
  const long long nc = P.ncell;
#pragma unroll
  for (int k = 0; k < FdaRing<C>::NF; ++k) r.v[slot(w)][k][f] = wplane(a, L::F_GPHI + k, nc)[cell];
}

// One block of the tiled gather: the tile and layer chunk bp, its
// parameter terms added to row (NPAR values).
template <class C>
__device__ inline void gather_tile_block(const AdjArgs<C>& a, const KParams& P, const BlockPos& bp,
                                         FdaRing<C>& ring, double* row) {
  const int tid = threadIdx.x;
  const int tx = tid % C::TX, ty = tid / C::TX;
  const int gx = bp.tx0 + tx, gy = bp.ty0 + ty;
  const bool own = gx < P.nx && (C::DIM == 2 || gy < P.ny);
  const int fc = (C::DIM == 3) ? (ty + 1) * C::LX + tx + 1 : tx + 1;
  double g[NPAR];
#pragma unroll
  for (int k = 0; k < NPAR; ++k) g[k] = 0.0;
  if (bp.w0 > 0)
    for (int f = tid; f < C::F; f += C::NT) fda_fill<C>(a, P, ring, bp, f, bp.w0 - 1);
  for (int f = tid; f < C::F; f += C::NT) fda_fill<C>(a, P, ring, bp, f, bp.w0);
  __syncthreads();
  for (int w = bp.w0; w < bp.w1; ++w) {
    if (w + 1 < P.nwn)
      for (int f = tid; f < C::F; f += C::NT) fda_fill<C>(a, P, ring, bp, f, w + 1);
    __syncthreads();
    if (own) {
      FdaLds<C> acc;
      acc.ring = &ring;
      acc.fc = fc;
      acc.w = w;
      const int cell = w * (int)P.area + ((C::DIM == 3) ? gy * P.nx + gx : gx);
      adj_gather_cell<C>(a, P, cell, false, g, acc);
    }
    __syncthreads();
  }
  block_sum_to<NPAR, true, C::NT>(g, row);
}

template <class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(4)))
    adj_gather_tile_kernel(AdjArgs<C> a, const KParams* __restrict__ kp, double* __restrict__ part, int ntx,
                           int nty, int chunk, int nblocks) {
  const KParams& P = *kp;
  __shared__ FdaRing<C> ring;
  StepArgs<typename C::S> sa;
  sa.ntx = ntx;
  sa.nty = nty;
  sa.chunk = chunk;
  sa.nblocks = nblocks;
  const int t = xcd_remap(blockIdx.x, nblocks);
  gather_tile_block<C>(a, P, block_pos_local<C>(sa, P, t), ring, part + (long long)t * NPAR);
}

// Which form the collide reverse takes, from the phase count and the number
// of tiles of the step geometry: for N >= 3 the tiled layer march below
// (fewer live registers than reading every neighbour's fields from global
// memory); for N = 2 the tiled form once the grid has TILED2_MIN_TILES tiles
// (about 512² cells), where it is faster; below that its blocks underfill the
// GPU and one thread per cell is faster; for N = 1 one thread per cell.  The
// batched kernels apply the same rule to each case, so batched and
// single-case sweeps stay bitwise equal.
constexpr long long TILED2_MIN_TILES = 512;
constexpr bool collide_reverse_tiled(int NP, long long tiles) {
  return NP >= 3 || (NP == 2 && tiles >= TILED2_MIN_TILES);
}

template <class C>
__global__ void __launch_bounds__(ADJ_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
    adj_collide_kernel(AdjArgs<C> a, const KParams* __restrict__ kp, double* __restrict__ part) {
  const KParams& P = *kp;
  double g[NPAR];
#pragma unroll
  for (int k = 0; k < NPAR; ++k) g[k] = 0.0;
  const int cell = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (cell < P.ncell) adj_collide_cell<C>(a, P, cell, g);
  block_sum<NPAR, true>(g, part);
}

// The collide reverse with its neighbour fields (phi_p, f_s, rho, u^{n-1}
// of the footprint, wall ghosts included) staged in the forward kernel's LDS
// ring: the block marches its tile along the wall-normal axis and fills the
// ring with the forward fill, from the moments of x^n (x^{n+1}'s lagged
// planes, or the recomputed work planes, laid out alike).  It holds the
// forward recompute and the whole reverse of a cell: capped at 256 registers
// (two waves per SIMD); the gather at 128.
template <class C>
struct NbLds {
  const Smem<C>* sm;
  int fc, w;
  __host__ __device__ void operator()(const KParams&, int i, typename C::R* phi, typename C::R& fs,
                                      typename C::R& rho, typename C::R* up) const {
    using Lt = typename C::L;
    const int s = slot(w + Lt::cw(i));
    const int f = fc + Lt::cl0(i) + (C::DIM == 3 ? Lt::cl1(i) * C::LX : 0);
#pragma unroll
    for (int p = 0; p < C::NP; ++p) phi[p] = sm->phi[s][p][f];
    fs = sm->fs[s][f];
    rho = sm->rho[s][f];
#pragma unroll
    for (int d = 0; d < C::DIM; ++d) up[d] = sm->u[s][d][f];
  }
};

// Fill arguments of the forward fill for the reverse step's x^n.
template <class C>
__host__ __device__ inline StepArgs<typename C::S> fill_args(const AdjArgs<C>& a, int ntx, int nty, int chunk,
                                                             int nblocks) {
  using S = typename C::S;
  // the recomputed moments (work planes M_PHI.., M_FS) stand in for the
  // moment planes phi_p.., f_s when x^{n+1} is not given: same order, type
  static_assert(sizeof(typename C::R) == sizeof(S), "work planes and state share the element type");
  static_assert(AdjLayout<C>::M_PHI == 0 && AdjLayout<C>::M_FS == C::A_FS, "moment plane order");
  StepArgs<S> sa;
  sa.pin = a.pin;
  sa.ain = a.ain;
  sa.mom = a.mom ? a.mom : reinterpret_cast<const S*>(a.work);
  sa.ntx = ntx;
  sa.nty = nty;
  sa.chunk = chunk;
  sa.nblocks = nblocks;
  return sa;
}

// One block of the tiled collide reverse: tile and chunk bp, parameter terms
// added to row (NPAR values).
template <class C>
__device__ inline void collide_tile_block(const AdjArgs<C>& a, const StepArgs<typename C::S>& sa, const KParams& P,
                                          const BlockPos& bp, Smem<C>& sm, double* row) {
  const int tid = threadIdx.x;
  const int tx = tid % C::TX, ty = tid / C::TX;
  const int gx = bp.tx0 + tx, gy = bp.ty0 + ty;
  const bool own = gx < P.nx && (C::DIM == 2 || gy < P.ny);
  double g[NPAR];
#pragma unroll
  for (int k = 0; k < NPAR; ++k) g[k] = 0.0;
  if (bp.w0 == 0) {
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(sa, P, sm, bp, f, 0);
    __syncthreads();
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(sa, P, sm, bp, f, -1);
  } else {
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(sa, P, sm, bp, f, bp.w0 - 1);
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(sa, P, sm, bp, f, bp.w0);
  }
  __syncthreads();
  for (int w = bp.w0; w < bp.w1; ++w) {
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(sa, P, sm, bp, f, w + 1);
    __syncthreads();
    if (own) {
      NbLds<C> nb;
      nb.sm = &sm;
      nb.fc = (C::DIM == 3) ? (ty + 1) * C::LX + tx + 1 : tx + 1;
      nb.w = w;
      const int cell = w * (int)P.area + ((C::DIM == 3) ? gy * P.nx + gx : gx);
      adj_collide_cell<C>(a, P, cell, g, nb);
    }
    __syncthreads();
  }
  block_sum_to<NPAR, true, C::NT>(g, row);
}

// The row of a block is its tile index (the block number after the XCD
// remap), in both tiled passes, so that a batched launch, whose remap spans
// many cases, fills the same rows in the same order.

template <class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2)))
    adj_collide_tile_kernel(AdjArgs<C> a, const KParams* __restrict__ kp, double* __restrict__ part, int ntx,
                            int nty, int chunk, int nblocks) {
  const KParams& P = *kp;
  __shared__ Smem<C> sm;
  const StepArgs<typename C::S> sa = fill_args<C>(a, ntx, nty, chunk, nblocks);
  const int t = xcd_remap(blockIdx.x, nblocks);
  collide_tile_block<C>(a, sa, P, block_pos_local<C>(sa, P, t), sm, part + (long long)t * NPAR);
}

template <class C>
__global__ void __launch_bounds__(ADJ_THREADS)
    adj_objective_kernel(AdjArgs<C> a, const KParams* __restrict__ kp, double* __restrict__ part) {
  using L = AdjLayout<C>;
  const KParams& P = *kp;
  double g[2] = {0.0, 0.0};
  const int cell = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (cell < P.ncell) {
    const long long nc = P.ncell;
    double psi = 0.0;
#pragma unroll
    for (int p = 0; p < C::NP; ++p)
      if (P.freezes[p]) psi += double(wplane(a, L::M_PHI + p, nc)[cell]);
    g[0] = double(wplane(a, L::M_FS, nc)[cell]) * psi;
    g[1] = psi;
  }
  block_sum<2, false>(g, part);
}

template <class C>
__global__ void __launch_bounds__(ADJ_THREADS)
    adj_seed_kernel(AdjArgs<C> a, const KParams* __restrict__ kp, double shift, double scale) {
  const KParams& P = *kp;
  const int cell = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (cell < P.ncell) adj_seed_cell<C>(a, P, cell, shift, scale);
}

template <class C>
__global__ void __launch_bounds__(ADJ_THREADS)
    adj_init_latent_kernel(AdjArgs<C> a, const KParams* __restrict__ kp, double* __restrict__ part) {
  const KParams& P = *kp;
  double g[NPAR];
#pragma unroll
  for (int k = 0; k < NPAR; ++k) g[k] = 0.0;
  const int cell = blockIdx.x * ADJ_THREADS + threadIdx.x;
  if (cell < P.ncell) adj_init_latent_cell<C>(a, P, cell, g);
  block_sum<NPAR, true>(g, part);
}

// Launchers.  pass: 0 moments, 1 collide, 2 gather, 3 seed gather,
// 4 objective partials, 5 seed (A = shift, B = scale), 6 initial-state
// latent term.
template <int DIM, int NP, typename S, typename R>
inline hipError_t launch_adjoint(int pass, const S* pin, const S* ain, const S* lpin, const S* lain, S* lpout,
                                 S* laout, const S* mom, void* work, const KParams& P, const KParams* dP,
                                 double* part, double A, double B, hipStream_t s) {
  using C = CfgOf<DIM, NP, S, R>;
  AdjArgs<C> a;
  a.pin = pin;
  a.ain = ain;
  a.lpin = lpin;
  a.lain = lain;
  a.lpout = lpout;
  a.laout = laout;
  a.mom = mom;
  a.work = static_cast<R*>(work);
  const int nb = (int)((P.ncell + ADJ_THREADS - 1) / ADJ_THREADS);
  const dim3 grid(nb), block(ADJ_THREADS);
  switch (pass) {
    case 0: hipLaunchKernelGGL((adj_moment_kernel<C>), grid, block, 0, s, a, dP); break;
    case 1:
      if constexpr (NP <= 2) {
        if (!collide_reverse_tiled(NP, step_geometry<C>(P).nblocks)) {
          hipLaunchKernelGGL((adj_collide_kernel<C>), grid, block, 0, s, a, dP, part);
          break;
        }
      }
      [[fallthrough]];
    case 2: {
      // the gradient rows of the buffer layout assume 128-cell rows and
      // chunks of at least two layers in 2D
      static_assert(DIM != 2 || (C::TX == 128 && C::TY == 1), "2D adjoint tile must be a 128-cell row");
      const Geometry g = step_geometry<C>(P);
      if (pass == 1)
        hipLaunchKernelGGL((adj_collide_tile_kernel<C>), dim3(g.nblocks), dim3(C::NT), 0, s, a, dP, part, g.ntx,
                           g.nty, g.chunk, g.nblocks);
      else
        hipLaunchKernelGGL((adj_gather_tile_kernel<C>), dim3(g.nblocks), dim3(C::NT), 0, s, a, dP, part, g.ntx,
                           g.nty, g.chunk, g.nblocks);
      break;
    }
    case 3: hipLaunchKernelGGL((adj_gather_kernel<C, true>), grid, block, 0, s, a, dP, part); break;
    case 4: hipLaunchKernelGGL((adj_objective_kernel<C>), grid, block, 0, s, a, dP, part); break;
    case 5: hipLaunchKernelGGL((adj_seed_kernel<C>), grid, block, 0, s, a, dP, A, B); break;
    case 6: hipLaunchKernelGGL((adj_init_latent_kernel<C>), grid, block, 0, s, a, dP, part); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lbf
