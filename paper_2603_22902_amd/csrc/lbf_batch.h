// Batched time step: many independent cases (different grid sizes and
// parameters, one phase count N) advance together, each pass one launch over
// all cases.  A block looks up its case in the pass's block-to-case map
// (stored after the case table), copies the case's parameter block into LDS
// and runs the same phase functions as the single-case kernels.  The result
// of each case is bitwise that of its single-case step: the per-cell
// arithmetic does not depend on the tile shape or on the batch.
#pragma once

#include <hip/hip_runtime.h>

#include "lbf_kernels.h"

namespace lbf {

// One case of a batch.  Buffer cur holds the state at even batch steps.
// pop_off, aux_off: the case's own two state buffers, as byte offsets from
// the base address the kernels take as an argument.  (A pointer read from
// the table would be generic to the compiler, which then emits flat memory
// instructions; those count against the LDS counter too, so every wait for
// an LDS read of the ring would also wait for the global traffic.  A
// kernel argument plus an offset is known to be global.)  soff, pop_bytes:
// where the case's state sits in a packed batch state (all cases' device
// states, each laid out as lbf_state_to_device writes it).
template <typename S>
struct BatchCase {
  const KParams* P;  // device copy of the case's parameter block
  long long pop_off[2], aux_off[2];
  long long soff, pop_bytes;
  int cur;
  int ntx, nty, chunk, nblocks;  // collide-pass geometry of this case
  int mblocks;                   // moments-pass blocks of this case
  int first_cblock, first_mblock;
  int map_m, map_c;  // the block-to-case maps, in ints from the table's start (same in every case)
};

// The case of block b of a pass: one entry of the pass's block-to-case map
// (written with the table), which the table's first case locates.  Two
// dependent scalar loads, where a binary search over the cases' first
// blocks took one per level.
template <typename S>
__device__ inline int batch_case(const BatchCase<S>* cs, int ncase, int b, bool collide) {
  const int* map = reinterpret_cast<const int*>(cs) + (collide ? cs[0].map_c : cs[0].map_m);
  return map[b];
}

__device__ inline void load_params(KParams& dst, const KParams* src) {
  static_assert(sizeof(KParams) % 4 == 0, "parameter block is copied as 32-bit words");
  const int* s = reinterpret_cast<const int*>(src);
  int* d = reinterpret_cast<int*>(&dst);
  for (int k = threadIdx.x; k < (int)(sizeof(KParams) / 4); k += blockDim.x) d[k] = s[k];
  __syncthreads();
}

// Pointers of a case's step: its own buffers at the given parity (src and
// dst are then both the base address of the offsets), or (PACKED) the
// case's slice of the packed batch states src -> dst.
template <typename S, bool PACKED>
__device__ inline void batch_io(const BatchCase<S>& bc, int parity, const char* src, char* dst, StepArgs<S>& a) {
  if constexpr (PACKED) {
    a.pin = reinterpret_cast<const S*>(src + bc.soff);
    a.ain = reinterpret_cast<const S*>(src + bc.soff + bc.pop_bytes);
    a.pout = reinterpret_cast<S*>(dst + bc.soff);
    a.aout = reinterpret_cast<S*>(dst + bc.soff + bc.pop_bytes);
  } else {
    const int in = bc.cur ^ parity;
    a.pin = reinterpret_cast<const S*>(src + bc.pop_off[in]);
    a.pout = reinterpret_cast<S*>(dst + bc.pop_off[1 - in]);
    a.ain = reinterpret_cast<const S*>(src + bc.aux_off[in]);
    a.aout = reinterpret_cast<S*>(dst + bc.aux_off[1 - in]);
  }
}

// Both passes take their work items (moment blocks of MOMENT_THREADS cells;
// collide tiles with their layer chunk) either one per block (PERSIST =
// false: item = blockIdx.x) or, in a persistent launch (a fixed grid, a
// multiple of 8), as item = blockIdx.x, blockIdx.x + gridDim.x, ... below
// nitems: each block keeps the items of one residue mod 8, so that the XCD
// remap of the item index still gives every XCD a contiguous range of
// tiles.  The two forms are separate kernels: the loop costs the collide
// pass registers (144 against 128 VGPRs for N = 3, one wave per SIMD less).
template <class C, bool PACKED>
__device__ __forceinline__ void batch_moment_item(const BatchCase<typename C::S>* __restrict__ cs, int ncase, int it,
                                         int parity, const char* __restrict__ src, char* __restrict__ dst,
                                         KParams& P) {
  using S = typename C::S;
  const int k = batch_case<S>(cs, ncase, it, false);
  const BatchCase<S>& bc = cs[k];
  load_params(P, bc.P);
  StepArgs<S> a;
  batch_io<S, PACKED>(bc, parity, src, dst, a);
  const int cell = (it - bc.first_mblock) * MOMENT_THREADS + threadIdx.x;
  if (cell < P.ncell) moment_cell<C>(a, P, cell);
}

template <class C, bool PACKED, bool PERSIST>
__global__ void __launch_bounds__(MOMENT_THREADS)
    batch_moment_kernel(const BatchCase<typename C::S>* __restrict__ cs, int ncase, int nitems, int parity,
                        const char* __restrict__ src, char* __restrict__ dst) {
  __shared__ KParams P;
  if constexpr (PERSIST) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
      if (it != (int)blockIdx.x) __syncthreads();  // every thread is done with the previous item's P
      batch_moment_item<C, PACKED>(cs, ncase, it, parity, src, dst, P);
    }
  } else {
    batch_moment_item<C, PACKED>(cs, ncase, blockIdx.x, parity, src, dst, P);
  }
}

template <class C, bool PACKED>
__device__ __forceinline__ void batch_collide_item(const BatchCase<typename C::S>* __restrict__ cs, int ncase, int Lg,
                                          int parity, const char* __restrict__ src, char* __restrict__ dst,
                                          KParams& P, Smem<C>& sm) {
  using S = typename C::S;
  const int k = batch_case<S>(cs, ncase, Lg, true);
  const BatchCase<S>& bc = cs[k];
  load_params(P, bc.P);
  StepArgs<S> a;
  batch_io<S, PACKED>(bc, parity, src, dst, a);
  a.mom = a.aout;
  a.mout = nullptr;
  a.mfield = 0;
  a.ntx = bc.ntx;
  a.nty = bc.nty;
  a.chunk = bc.chunk;
  a.nblocks = bc.nblocks;
  const BlockPos bp = block_pos_local<C>(a, P, Lg - bc.first_cblock);
  const int tid = threadIdx.x;
  if (bp.w0 == 0) {
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(a, P, sm, bp, f, 0);
    __syncthreads();
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(a, P, sm, bp, f, -1);
  } else {
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(a, P, sm, bp, f, bp.w0 - 1);
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(a, P, sm, bp, f, bp.w0);
  }
  __syncthreads();
  for (int w = bp.w0; w < bp.w1; ++w) {
    for (int f = tid; f < C::F; f += C::NT) fill_layer_cell<C>(a, P, sm, bp, f, w + 1);
    __syncthreads();
    if (w == 0 || w == P.nwn - 1)
      process_cell<C, false, true>(a, P, sm, bp, tid, w);
    else
      process_cell<C, false, false>(a, P, sm, bp, tid, w);
    __syncthreads();
  }
}

template <class C, bool PACKED, bool PERSIST>
__global__ void __launch_bounds__(C::NT)
    batch_collide_kernel(const BatchCase<typename C::S>* __restrict__ cs, int ncase, int nitems, int parity,
                         const char* __restrict__ src, char* __restrict__ dst) {
  __shared__ KParams P;
  __shared__ Smem<C> sm;
  if constexpr (PERSIST) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
      if (it != (int)blockIdx.x) __syncthreads();  // the previous item's P and ring are no longer read
      batch_collide_item<C, PACKED>(cs, ncase, xcd_remap(it, nitems), parity, src, dst, P, sm);
    }
  } else {
    batch_collide_item<C, PACKED>(cs, ncase, xcd_remap(blockIdx.x, nitems), parity, src, dst, P, sm);
  }
}

// 2D row tiles the batch can use (the autotuner picks one per phase count).
constexpr int BATCH_TILES[3] = {64, 128, 256};

// Geometry of one case for a row tile of tx cells: ntx tiles per row and a
// chunk of layers chosen so that the case gets about `target` blocks (at
// least two layers per chunk).
inline void batch_geometry(const KParams& P, int tx, long long target, int& ntx, int& chunk, int& nblocks) {
  ntx = (P.nx + tx - 1) / tx;
  long long c = ((long long)P.nwn * ntx + target - 1) / (target > 0 ? target : 1);
  if (c < 2) c = 2;
  if (c > P.nwn) c = P.nwn;
  chunk = (int)c;
  nblocks = (int)((long long)ntx * ((P.nwn + chunk - 1) / chunk));
}

// Blocks of kernel k (blockDim threads, static LDS only) that the whole GPU
// holds at once, rounded down to a multiple of 8 (one per XCD); 0 on error.
inline int resident_blocks(const void* k, int block) {
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, 0) != hipSuccess) return 0;
  return (per_cu * cus) / 8 * 8;
}

// Grid of a pass over nitems items.  grid = 0: one block per item; grid > 0
// (a multiple of 8): that many persistent blocks; grid < 0: as many
// persistent blocks as the GPU holds at once (the kernel's resident count).
// Never more blocks than items.
inline int batch_grid(int resident, int nitems, int grid) {
  const int g = grid > 0 ? grid : (grid < 0 ? resident : 0);
  return (g >= 8 && g < nitems) ? g : nitems;
}

// The resident block count is queried once per kernel, on its first launch
// with grid < 0; nitems = 0 makes only that query (no launch), so that it
// need not happen during a graph capture.
template <class C, bool PACKED>
inline hipError_t launch_collide_batch(const BatchCase<typename C::S>* cs, int ncase, int nitems, int parity,
                                       const char* src, char* dst, int grid, hipStream_t s) {
  if (grid == 0) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL((batch_collide_kernel<C, PACKED, false>), dim3(nitems), dim3(C::NT), 0, s, cs, ncase, nitems,
                       parity, src, dst);
    return hipGetLastError();
  }
  int resident = 0;
  if (grid < 0) {
    static const int r =
        resident_blocks(reinterpret_cast<const void*>(&batch_collide_kernel<C, PACKED, true>), C::NT);
    resident = r;
  }
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL((batch_collide_kernel<C, PACKED, true>), dim3(batch_grid(resident, nitems, grid)), dim3(C::NT),
                     0, s, cs, ncase, nitems, parity, src, dst);
  return hipGetLastError();
}

template <int NP, typename S, typename R, bool PACKED>
inline hipError_t launch_batch_t(int pass, int variant, const BatchCase<S>* cs, int ncase, int nitems, int parity,
                                 const char* src, char* dst, int grid, hipStream_t s) {
  if (pass == 0) {
    using C = Cfg<2, NP, S, R, 128, 1>;
    if (grid == 0) {
      if (nitems <= 0) return hipSuccess;
      hipLaunchKernelGGL((batch_moment_kernel<C, PACKED, false>), dim3(nitems), dim3(MOMENT_THREADS), 0, s, cs,
                         ncase, nitems, parity, src, dst);
      return hipGetLastError();
    }
    int resident = 0;
    if (grid < 0) {
      static const int r =
          resident_blocks(reinterpret_cast<const void*>(&batch_moment_kernel<C, PACKED, true>), MOMENT_THREADS);
      resident = r;
    }
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL((batch_moment_kernel<C, PACKED, true>), dim3(batch_grid(resident, nitems, grid)),
                       dim3(MOMENT_THREADS), 0, s, cs, ncase, nitems, parity, src, dst);
    return hipGetLastError();
  }
  switch (variant) {
    case 0: return launch_collide_batch<Cfg<2, NP, S, R, 64, 1>, PACKED>(cs, ncase, nitems, parity, src, dst, grid, s);
    case 1: return launch_collide_batch<Cfg<2, NP, S, R, 128, 1>, PACKED>(cs, ncase, nitems, parity, src, dst, grid, s);
    case 2: return launch_collide_batch<Cfg<2, NP, S, R, 256, 1>, PACKED>(cs, ncase, nitems, parity, src, dst, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// pass 0: moments, 1: collide; variant indexes BATCH_TILES.  packed: the
// step reads the packed batch state src and writes dst; else src = dst =
// the base address of the cases' own-buffer offsets.  grid as batch_grid:
// 0 one block per item, else persistent blocks striding over the items.
template <int NP, typename S, typename R>
inline hipError_t launch_batch(int pass, int variant, const void* cases, int ncase, int nitems, int parity,
                               const void* src, void* dst, bool packed, int grid, hipStream_t s) {
  const auto* cs = static_cast<const BatchCase<S>*>(cases);
  if (!src || !dst) return hipErrorInvalidValue;
  if (packed)
    return launch_batch_t<NP, S, R, true>(pass, variant, cs, ncase, nitems, parity, static_cast<const char*>(src),
                                          static_cast<char*>(dst), grid, s);
  return launch_batch_t<NP, S, R, false>(pass, variant, cs, ncase, nitems, parity, static_cast<const char*>(src),
                                         static_cast<char*>(dst), grid, s);
}

}  // namespace lbf
