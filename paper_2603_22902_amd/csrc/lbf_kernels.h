// HIP kernels of the coupled LB solver and their launchers.
//
//   moment_kernel   phi_p^n, f_s^n of every cell (first pass of a step)
//   collide_kernel  finite differences, sources, collisions and push
//                   streaming (or, with MOMENTS, one macroscopic field at
//                   the current time level)
//   init_kernel     equilibrium start from phi, T (and optionally u, p)
//   diag_kernel     float64 conservation sums, two deterministic passes
//   widen_kernel    float32 -> float64 copy of one plane for read-back
#pragma once

#include <hip/hip_runtime.h>

#include "lbf_step.h"

namespace lbf {

// Tile shapes (by arithmetic type, which is also the LDS type).  2D: one
// row of 128 cells per block.  3D: 64 x 8 cells in float32 (a wave covers
// one 64-cell row, i.e. two whole 128-byte lines per plane; 512 threads = one
// block of 8 waves per CU at two waves per SIMD); 32 x 4 in float64, whose
// LDS ring is twice as large.  Measured on the 192^3 workload, float32:
// 64 x 8 1.57 ms, 64 x 4 1.58 ms, 192 x 1 1.58 ms, 128 x 2 1.91 ms,
// 32 x 8 2.02 ms, 32 x 4 2.26 ms per collide launch.
template <int DIM, typename R>
struct Tile;
template <typename R>
struct Tile<2, R> {
  static constexpr int TX = 128, TY = 1;
};
template <>
struct Tile<3, float> {
  static constexpr int TX = 64, TY = 8;
};
template <>
struct Tile<3, double> {
  static constexpr int TX = 32, TY = 4;
};

template <int DIM, int NP, typename S, typename R>
using CfgOf = Cfg<DIM, NP, S, R, Tile<DIM, R>::TX, Tile<DIM, R>::TY>;

// ---------------------------------------------------------------------------
// One time step: moments pass, then collide pass
// ---------------------------------------------------------------------------
constexpr int MOMENT_THREADS = 256;

template <class C>
__global__ void __launch_bounds__(MOMENT_THREADS)
    moment_kernel(const typename C::S* __restrict__ pin, const typename C::S* __restrict__ ain,
                  typename C::S* __restrict__ aout, StepArgs<typename C::S> a,
                  const KParams* __restrict__ kp) {
  const KParams& P = *kp;
  a.pin = pin;
  a.ain = ain;
  a.aout = aout;
  const int cell = blockIdx.x * MOMENT_THREADS + threadIdx.x;
  if (cell < P.ncell) moment_cell<C>(a, P, cell);
}

// The buffers are separate kernel parameters so that the compiler knows
// they are global memory (global rather than flat loads and stores).  The
// parameter block is a separate restrict pointer too: no store of the
// kernel can alias it, so its fields are read with scalar loads.
template <class C, bool MOMENTS>
__global__ void __launch_bounds__(C::NT)
    collide_kernel(const typename C::S* __restrict__ pin, typename C::S* __restrict__ pout,
                   const typename C::S* __restrict__ ain, typename C::S* __restrict__ aout,
                   const typename C::S* __restrict__ mom, double* __restrict__ mout,
                   StepArgs<typename C::S> a, const KParams* __restrict__ kp) {
  const KParams& P = *kp;
  a.pin = pin;
  a.pout = pout;
  a.ain = ain;
  a.aout = aout;
  a.mom = mom;
  a.mout = mout;
  __shared__ Smem<C> sm;
  const BlockPos bp = block_pos<C>(a, P, blockIdx.x);
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
      process_cell<C, MOMENTS, true>(a, P, sm, bp, tid, w);
    else
      process_cell<C, MOMENTS, false>(a, P, sm, bp, tid, w);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Initial state: f_l = 1 where T > T_melt else 0, rho H from eq. (H),
// populations at equilibrium, lagged fields (phi, f_s, u, 0, 0).
// fields: phi [N][cells], T [cells], then u [DIM][cells] if has_u, then
// p [cells] if has_p (float64).
// ---------------------------------------------------------------------------
template <int DIM, int NP, typename R>
__host__ __device__ inline void init_cell(const KParams& P, const double* fields, int has_u,
                                          int has_p, R* pop, R* aux, long long cell) {
  // R here is the storage type; the equilibria are formed in float64.
  using L = Lat<DIM>;
  constexpr int Q = L::Q;
  const long long nc = P.ncell;
  double phi[NP];
  for (int p = 0; p < NP; ++p) phi[p] = fields[p * nc + cell];
  const double T = fields[NP * nc + cell];
  double u[3] = {0, 0, 0};
  long long off = (NP + 1) * nc;
  if (has_u) {
    for (int d = 0; d < DIM; ++d) u[d] = fields[off + d * nc + cell];
    off += DIM * nc;
  }
  const double pr = has_p ? fields[off + cell] : 0.0;
  const double fl = (T > P.T_melt) ? 1.0 : 0.0;
  double rs = 0, rl = 0, cs = 0, cl = 0, Lv = 0;
  for (int p = 0; p < NP; ++p) {
    rs += phi[p] * P.rho_s[p];
    rl += phi[p] * P.rho_l[p];
    cs += phi[p] * P.cp_s[p];
    cl += phi[p] * P.cp_l[p];
    Lv += phi[p] * P.rho_l[p] * P.latent[p];
  }
  const double rhoH = (fl <= 0.0) ? rs * cs * T : rl * cl * T + Lv;
  const double fs = 1.0 - fl;
  double rho = 0, cp = 0;
  for (int p = 0; p < NP; ++p) {
    rho += fs * phi[p] * P.rho_s[p] + (1.0 - fs) * phi[p] * P.rho_l[p];
    cp += fs * phi[p] * P.cp_s[p] + (1.0 - fs) * phi[p] * P.cp_l[p];
  }
  const double rhocp = rho * cp;
  double uu = 0.0;
  for (int d = 0; d < DIM; ++d) uu += u[d] * u[d];
  const double w0 = wgt<double, DIM>(0);
  for (int i = 0; i < Q; ++i) {
    double cu = 0.0;
    for (int d = 0; d < DIM; ++d) cu += L::c(i, d) * u[d];
    const double wi = wgt<double, DIM>(i);
    const double si = wi * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    const double fe = (i == 0) ? 3.0 * pr * (w0 - 1.0) + rho * si : 3.0 * pr * wi + rho * si;
    pop[i * nc + cell] = R(fe);
    for (int p = 0; p < NP; ++p) pop[((1 + p) * Q + i) * nc + cell] = R(wi * phi[p] * (1.0 + 3.0 * cu));
    const double he = (i == 0) ? rhoH - P.E_ref * T + w0 * (P.E_ref * T - 1.5 * rhocp * T * uu)
                               : wi * (P.E_ref * T + rhocp * T * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    pop[((NP + 1) * Q + i) * nc + cell] = R(he);
  }
  for (int p = 0; p < NP; ++p) aux[p * nc + cell] = R(phi[p]);
  aux[NP * nc + cell] = R(fs);
  for (int d = 0; d < DIM; ++d) aux[(NP + 1 + d) * nc + cell] = R(u[d]);
  aux[(NP + 1 + DIM) * nc + cell] = R(0);
  aux[(NP + 2 + DIM) * nc + cell] = R(0);
}

template <int DIM, int NP, typename R>
__global__ void init_kernel(const KParams* __restrict__ kp, const double* __restrict__ fields, int has_u,
                            int has_p, R* __restrict__ pop, R* __restrict__ aux) {
  const KParams& P = *kp;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < P.ncell; c += stride)
    init_cell<DIM, NP, R>(P, fields, has_u, has_p, pop, aux, c);
}

// ---------------------------------------------------------------------------
// Diagnostics: per-cell moments and inversion, then float64 sums.
// Values: [0,N) mass, [N,2N) solid volume, [2N,3N) volume, 3N sum rhoH,
// 3N+1 max |sum phi - 1|, 3N+2 sum f_s psi, 3N+3 non-finite flag.
// ---------------------------------------------------------------------------
template <int NP>
struct DiagN {
  static constexpr int NV = 3 * NP + 4;
};

template <int DIM, int NP, typename S, typename R>
__host__ __device__ inline void diag_cell(const KParams& P, const S* pop, const S* aux,
                                          long long cell, double* acc) {
  constexpr int Q = Lat<DIM>::Q;
  const long long nc = P.ncell;
  // phi_p and f_s exactly as the moments pass forms and stores them
  const double idiv = 1.0 / (1.0 - 0.5 * double(aux[(NP + 1 + DIM) * nc + cell]));
  const double qv = double(aux[(NP + 2 + DIM) * nc + cell]);
  double phi[NP];
  for (int p = 0; p < NP; ++p) {
    MomSum<S> sum;
    for (int i = 0; i < Q; ++i) sum.add(pop[((1 + p) * Q + i) * nc + cell]);
    phi[p] = double(S(sum.value() * idiv));
  }
  double sh = 0.0;
  for (int i = 0; i < Q; ++i) sh += double(pop[((NP + 1) * Q + i) * nc + cell]);
  const double rhoH = sh + 0.5 * qv;
  double T, fl;
  invert<NP>(P, phi, rhoH, T, fl);
  const double fs = double(S(1.0 - fl));
  double s = 0.0, psi = 0.0;
  bool bad = !(rhoH == rhoH) || rhoH - rhoH != 0.0;
  for (int p = 0; p < NP; ++p) {
    const double ph = phi[p];
    acc[p] += ph * (fs * P.rho_s[p] + (1.0 - fs) * P.rho_l[p]);
    acc[NP + p] += fs * ph;
    acc[2 * NP + p] += ph;
    s += ph;
    if (P.freezes[p]) psi += ph;
    if (!(ph == ph) || ph - ph != 0.0) bad = true;
  }
  acc[3 * NP] += rhoH;
  const double e = s > 1.0 ? s - 1.0 : 1.0 - s;
  if (e > acc[3 * NP + 1] || !(e == e)) acc[3 * NP + 1] = e;
  acc[3 * NP + 2] += fs * psi;
  if (bad) acc[3 * NP + 3] = 1.0;
}

constexpr int DIAG_THREADS = 256;
constexpr int DIAG_WAVES = DIAG_THREADS / 64;

// Combine of two partial diagnostics: maxima (with NaN kept) for the
// largest |sum phi - 1| and the non-finite flag, sums for the rest.
template <int NP>
__device__ inline double diag_combine(int k, double a, double b) {
  if (k == 3 * NP + 1 || k == 3 * NP + 3) return (a > b || !(a == a)) ? a : b;
  return a + b;
}

// Block reduction of NV values per thread: a butterfly over the 64 lanes of
// each wavefront (cross-lane shuffles, no barrier), then one value per wave
// through LDS, combined by the first wave in wave order.  The order of the
// combines is fixed, so the result is deterministic.  Thread 0 returns the
// block's values in v.
template <int NP>
__device__ inline void diag_block_reduce(double* v, double (*red)[DIAG_WAVES]) {
  constexpr int NV = DiagN<NP>::NV;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] = diag_combine<NP>(k, v[k], __shfl_xor(v[k], off, 64));
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wave] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double a = red[k][0];
#pragma unroll
      for (int w = 1; w < DIAG_WAVES; ++w) a = diag_combine<NP>(k, a, red[k][w]);
      v[k] = a;
    }
}

template <int DIM, int NP, typename S, typename R>
__global__ void __launch_bounds__(DIAG_THREADS)
    diag_kernel(const KParams* __restrict__ kp, const S* __restrict__ pop, const S* __restrict__ aux,
                double* __restrict__ part) {
  const KParams& P = *kp;
  constexpr int NV = DiagN<NP>::NV;
  __shared__ double red[NV][DIAG_WAVES];
  double acc[NV];
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < P.ncell; c += stride)
    diag_cell<DIM, NP, S, R>(P, pop, aux, c, acc);
  diag_block_reduce<NP>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) part[(long long)blockIdx.x * NV + k] = acc[k];
}

template <int NP>
__global__ void __launch_bounds__(DIAG_THREADS) diag_final_kernel(const double* part, int nparts,
                                                                  double inv_area, double* out) {
  constexpr int NV = DiagN<NP>::NV;
  __shared__ double red[NV][DIAG_WAVES];
  double acc[NV];
  for (int k = 0; k < NV; ++k) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nparts; b += DIAG_THREADS) a = diag_combine<NP>(k, a, part[(long long)b * NV + k]);
    acc[k] = a;
  }
  diag_block_reduce<NP>(acc, red);
  if (threadIdx.x == 0) {
    for (int k = 0; k < NV; ++k) out[k] = acc[k];
    out[3 * NP + 2] = acc[3 * NP + 2] * inv_area;
  }
}

template <typename R>
__global__ void widen_kernel(const R* in, double* out, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    out[k] = double(in[k]);
}

// ---------------------------------------------------------------------------
// Launch geometry and launchers
// ---------------------------------------------------------------------------
struct Geometry {
  int ntx, nty, chunk, nblocks, threads;
};

template <class C>
inline Geometry step_geometry(const KParams& P) {
  Geometry g;
  g.ntx = (P.nx + C::TX - 1) / C::TX;
  g.nty = (C::DIM == 3) ? (P.ny + C::TY - 1) / C::TY : 1;
  const long long ntiles = (long long)g.ntx * g.nty;
  // Aim for about 4608 blocks in 3D (18 per CU) and 4096 in 2D: many short
  // chunks balance the CUs better than a few long ones.  A chunk never drops
  // below 3 layers in 3D and 2 in 2D (each chunk re-reads two extra layers).
  const long long target = (C::DIM == 3) ? 4608 : 4096;
  long long chunk = (P.nwn * ntiles + target - 1) / target;
  const long long cmin = (C::DIM == 3) ? 3 : 2;
  if (chunk < cmin) chunk = cmin;
  if (chunk > P.nwn) chunk = P.nwn;
  g.chunk = (int)chunk;
  g.nblocks = (int)(ntiles * ((P.nwn + chunk - 1) / chunk));
  g.threads = C::NT;
  return g;
}

// Moments pass into the first N + 1 planes of a.aout (passes & 1), then
// the collide pass, which reads them through a.mom (passes & 2).  In
// moments mode a.aout is only used as that scratch and a.pout is not
// touched.
template <int DIM, int NP, typename S, typename R>
inline hipError_t launch_step(StepArgs<S> a, const KParams& hostP, const KParams* dP, hipStream_t s,
                              bool moments, int passes) {
  using C = CfgOf<DIM, NP, S, R>;
  const Geometry g = step_geometry<C>(hostP);
  a.ntx = g.ntx;
  a.nty = g.nty;
  a.chunk = g.chunk;
  a.nblocks = g.nblocks;
  a.mom = a.aout;
  const int mb = (int)((hostP.ncell + MOMENT_THREADS - 1) / MOMENT_THREADS);
  // One cell per thread (57 VGPRs, eight waves per SIMD): the compensated
  // float32 sums of the moments hide their latency behind many waves.  A
  // four-cells-per-thread variant with 16-byte loads ran at one wave per
  // SIMD and took 670 us against 552 us on the 192^3 workload.
  if (passes & 1)
    hipLaunchKernelGGL((moment_kernel<C>), dim3(mb), dim3(MOMENT_THREADS), 0, s, a.pin, a.ain, a.aout, a, dP);
  if (!(passes & 2)) return hipGetLastError();
  if (moments)
    hipLaunchKernelGGL((collide_kernel<C, true>), dim3(g.nblocks), dim3(g.threads), 0, s, a.pin,
                       a.pout, a.ain, a.aout, a.mom, a.mout, a, dP);
  else
    hipLaunchKernelGGL((collide_kernel<C, false>), dim3(g.nblocks), dim3(g.threads), 0, s, a.pin,
                       a.pout, a.ain, a.aout, a.mom, a.mout, a, dP);
  return hipGetLastError();
}

inline int grid_for(long long n, int threads, int cap) {
  long long b = (n + threads - 1) / threads;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

template <int DIM, int NP, typename R>
inline hipError_t launch_init(const KParams& P, const KParams* dP, const double* fields, int has_u,
                              int has_p, R* pop, R* aux, hipStream_t s) {
  hipLaunchKernelGGL((init_kernel<DIM, NP, R>), dim3(grid_for(P.ncell, 256, 65536)), dim3(256), 0,
                     s, dP, fields, has_u, has_p, pop, aux);
  return hipGetLastError();
}

static_assert(DIAG_THREADS == 256, "diag_blocks assumes 256-thread blocks");

template <int DIM, int NP, typename S, typename R>
inline hipError_t launch_diag(const KParams& P, const KParams* dP, const S* pop, const S* aux,
                              double* part, double* out, hipStream_t s) {
  const int nb = diag_blocks(P.ncell);
  hipLaunchKernelGGL((diag_kernel<DIM, NP, S, R>), dim3(nb), dim3(DIAG_THREADS), 0, s, dP, pop, aux,
                     part);
  hipLaunchKernelGGL((diag_final_kernel<NP>), dim3(1), dim3(DIAG_THREADS), 0, s, part, nb,
                     1.0 / double(P.area), out);
  return hipGetLastError();
}

template <typename R>
inline hipError_t launch_widen(const R* in, double* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL((widen_kernel<R>), dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace lbf
