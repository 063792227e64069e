// The coupled-LB time step of arXiv:2603.22902, Sec. 3, as two HIP kernels:
// a streaming moments pass and a collide pass of barrier-separated phases.
//
// Storage (structure of arrays, x fastest): populations
// pop[(lattice*Q + i)*ncell + cell], lattice 0 = f, 1..N = g_p, N+1 = h,
// holding post-stream values (the state at the start of a step); lagged
// fields aux[k*ncell + cell] = phi_p^{n-1} (N), f_s^{n-1}, u^{n-1} (DIM),
// D^{n-1} (velocity divergence used by the previous step's sources) and
// q^{n-1} = (rho C_p T D)^{n-1}.  A step reads buffers "in" and writes "out"
// (push streaming: each cell writes its post-collision values to x + c_i).
//
// Moments pass (one thread per cell): phi_p^n and f_s^n of every cell from
// its populations, written into planes 0..N of "out" aux, where the next
// step finds them as its lagged phi_p^{n-1}, f_s^{n-1}.  The finite
// differences of the collide pass then read 1 + N planes per neighbour
// instead of summing (N + 1) Q populations of every halo cell.
//
// Collide pass: a block owns a lateral tile of TX (x TY in 3D) cells and
// marches along the wall-normal axis (y in 2D, z in 3D) over a chunk of
// layers.  An LDS ring of three layers holds, for the tile plus a one-cell
// lateral halo, the fields the finite differences need (phi_p, f_s, rho,
// u^{n-1}); ghost layers outside the wall-normal faces are derived from
// the boundary layer in LDS.  Each cell's own rho H and T are recomputed
// from the h populations it loads for its collision.
//
// Every phase is a __host__ __device__ function of an explicit thread index
// so that the same code also runs in the host emulator used by the CPU
// tests; the device kernel and the emulator only differ in how they
// sequence the phases around the block barriers.
#pragma once

#include <math.h>

#include "lbf_lattice.h"

namespace lbf {

// S: storage type of populations and lagged fields; R: arithmetic type.
template <int DIM_, int NP_, typename S_, typename R_, int TX_, int TY_>
struct Cfg {
  static constexpr int DIM = DIM_, NP = NP_, TX = TX_, TY = TY_;
  using S = S_;
  using R = R_;
  using L = Lat<DIM_>;
  static constexpr int Q = L::Q;
  static constexpr int NT = TX * TY;
  static constexpr int LX = TX + 2;
  static constexpr int LY = (DIM == 3) ? TY + 2 : 1;
  static constexpr int F = LX * LY;  // footprint cells per layer
  static constexpr int NAUX = NP + DIM + 3;
  static constexpr int A_FS = NP, A_U = NP + 1, A_DIV = NP + 1 + DIM, A_Q = NP + 2 + DIM;
  static_assert(DIM == 3 || TY == 1, "2D tiles are one row of cells");
};

template <class C>
struct Smem {
  typename C::R phi[3][C::NP][C::F];
  typename C::R fs[3][C::F];
  typename C::R rho[3][C::F];
  typename C::R u[3][C::DIM][C::F];
};

template <typename S>
struct StepArgs {
  const S* pin;
  S* pout;
  const S* ain;
  S* aout;
  const S* mom;  // phi_p^n, f_s^n planes (the first N + 1 planes of aout)
  double* mout;  // moments mode: one float64 plane
  int mfield;    // moments mode: field id (phi_p, rhoH, T, f_l, rho, u, p, mdot)
  int ntx, nty;  // lateral tiles
  int chunk;     // layers per block
  int nblocks;
};

struct BlockPos {
  int tx0, ty0, w0, w1;
};

__host__ __device__ inline int imod(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}
__host__ __device__ inline int slot(int w) { return imod(w, 3); }
// Face attributes by a run-time face index without indexing the parameter
// block dynamically (which would force it into scratch memory).
__host__ __device__ inline int face_flow(const KParams& P, int f) { return f == 0 ? P.flow_bc[0] : P.flow_bc[1]; }
__host__ __device__ inline int face_therm(const KParams& P, int f) { return f == 0 ? P.therm_bc[0] : P.therm_bc[1]; }
__host__ __device__ inline double face_T(const KParams& P, int f) { return f == 0 ? P.T_face[0] : P.T_face[1]; }

// Start of plane k of a structure-of-arrays buffer (uniform across a wave,
// so the offset stays in scalar registers and cells index it in 32 bits).
template <typename T>
__host__ __device__ inline T* plane(T* base, long long k, long long nc) { return base + k * nc; }

// Periodic wrap of a coordinate at most one period outside [0, n).
__host__ __device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// Periodic wrap of a footprint coordinate (tiles wider than the domain
// reach further out).
__host__ __device__ inline int wrapf(int v, int n) {
  v = wrap1(v, n);
  return (v < 0 || v >= n) ? imod(v, n) : v;
}

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of logical blocks so that neighbouring tiles share an L2.
__host__ __device__ inline int xcd_remap(int b, int nb) {
  const int q = nb / 8, r = nb % 8;
  const int x = b % 8, k = b / 8;
  return x * q + (x < r ? x : r) + k;
}

// Tile and layer chunk of logical block Lg of one grid.
template <class C>
__host__ __device__ inline BlockPos block_pos_local(const StepArgs<typename C::S>& a, const KParams& P,
                                                    int Lg) {
  const int ntiles = a.ntx * a.nty;
  const int chunk_id = Lg / ntiles, tile = Lg % ntiles;
  BlockPos bp;
  bp.tx0 = (tile % a.ntx) * C::TX;
  bp.ty0 = (tile / a.ntx) * C::TY;
  bp.w0 = chunk_id * a.chunk;
  const int w1 = bp.w0 + a.chunk;
  bp.w1 = w1 < P.nwn ? w1 : P.nwn;
  return bp;
}

template <class C>
__host__ __device__ inline BlockPos block_pos(const StepArgs<typename C::S>& a, const KParams& P,
                                              int b) {
  return block_pos_local<C>(a, P, xcd_remap(b, a.nblocks));
}

// Mixture law, eq. (eq2).
template <typename R, int NP>
__host__ __device__ inline R mixture(const R* phi, R fs, const double* xs, const double* xl) {
  R x = R(0);
#pragma unroll
  for (int p = 0; p < NP; ++p) x += fs * phi[p] * R(xs[p]) + (R(1) - fs) * phi[p] * R(xl[p]);
  return x;
}

// Enthalpy inversion, eq. (H), always in float64.  Solid and liquid states
// are the eq. (eq2) mixtures at f_s = 1 and 0, the volumetric latent heat is
// sum_p phi_p rho_p^l L_p, solidus = liquidus = T_melt; an empty mushy range
// (no freezing phase present) counts as liquid.
template <int NP, typename R>
__host__ __device__ inline void invert(const KParams& P, const R* phi, double rhoH, double& T,
                                       double& fl) {
  double rs = 0, rl = 0, cs = 0, cl = 0, Lv = 0;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const double ph = double(phi[p]);
    rs += ph * P.rho_s[p];
    rl += ph * P.rho_l[p];
    cs += ph * P.cp_s[p];
    cl += ph * P.cp_l[p];
    Lv += ph * P.rho_l[p] * P.latent[p];
  }
  const double Tm = P.T_melt;
  const double Es = rs * cs * Tm;
  const double El = rl * cl * Tm + Lv;
  if (rhoH < Es) {
    fl = 0.0;
    T = rhoH / (rs * cs);
  } else if (rhoH > El) {
    fl = 1.0;
    T = Tm + (rhoH - El) / (rl * cl);
  } else {
    fl = (El > Es) ? (rhoH - Es) / (El - Es) : 1.0;
    T = Tm;
  }
}

// Own rho H = sum_i h_i + q^{n-1}/2 (float64) of a cell from its loaded h
// populations, and T, f_l by eq. (H).
template <class C>
__host__ __device__ inline double own_enthalpy(const KParams& P, const typename C::R* phi,
                                               const typename C::R* hpop, typename C::R qv,
                                               double& T, double& fl) {
  double sh = 0.0;
#pragma unroll
  for (int i = 0; i < C::Q; ++i) sh += double(hpop[i]);
  const double rhoH = sh + 0.5 * double(qv);
  invert<C::NP>(P, phi, rhoH, T, fl);
  return rhoH;
}

__host__ __device__ inline double gprime(double x) { return 2.0 * x * (1.0 - x) * (1.0 - 2.0 * x); }
__host__ __device__ inline float gprime(float x) { return 2.0f * x * (1.0f - x) * (1.0f - 2.0f * x); }

// ---------------------------------------------------------------------------
// Moments pass for one cell: phi_p = sum_i g_{i,p} / (1 - D^{n-1}/2),
// rho H = sum_i h_i + q^{n-1}/2, f_s = 1 - f_l from eq. (H).  phi_p is the
// zeroth moment every equilibrium g^eq is built from, so its rounding is
// what the collision adds to or removes from a phase's mass each step; a
// plain float32 sum of Q values rounds Q - 1 times where the stored plane
// rounds once (measured on the 1000:1 droplet after 100 steps against the
// float64 oracle: phi 3e-6 -> 1.2e-6, T 5.7e-5 -> 1.5e-5).  With float32
// storage the sum is therefore compensated (MomSum: the two-sum of each
// addition's rounding error kept in a second float, combined in float64 at
// the end), which keeps the register footprint of a float32 sum; float64
// storage sums in float64.  The division runs in float64.
// Cell indices are 32-bit (the host limits a grid to 2^30 cells); plane
// offsets k * ncell are formed in 64-bit once per plane.
// ---------------------------------------------------------------------------
template <typename ST>
struct MomSum;
template <>
struct MomSum<float> {
  float s = 0.0f, c = 0.0f;
  __host__ __device__ void add(float x) {
    const float t = s + x;
    const float z = t - s;
    c += (s - (t - z)) + (x - z);
    s = t;
  }
  __host__ __device__ double value() const { return double(s) + double(c); }
};
template <>
struct MomSum<double> {
  double s = 0.0;
  __host__ __device__ void add(double x) { s += x; }
  __host__ __device__ double value() const { return s; }
};

template <class C>
__host__ __device__ inline void moment_cell(const StepArgs<typename C::S>& a, const KParams& P,
                                            int cell) {
  using ST = typename C::S;
  constexpr int Q = C::Q, NP = C::NP;
  const long long nc = P.ncell;
  const ST* __restrict__ pin = a.pin;
  const ST* __restrict__ ain = a.ain;
  ST* __restrict__ aout = a.aout;
  const double div = double(plane(ain, C::A_DIV, nc)[cell]);
  const double qv = double(plane(ain, C::A_Q, nc)[cell]);
  const double idiv = 1.0 / (1.0 - 0.5 * div);
  // phi_p as stored (the value the collide pass and the inversion see)
  double phi[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    MomSum<ST> sum;
#pragma unroll
    for (int i = 0; i < Q; ++i) sum.add(plane(pin, (1 + p) * Q + i, nc)[cell]);
    phi[p] = double(ST(sum.value() * idiv));
  }
  double sh = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) sh += double(plane(pin, (NP + 1) * Q + i, nc)[cell]);
  const double rhoH = sh + 0.5 * qv;
  double T, fl;
  invert<NP>(P, phi, rhoH, T, fl);
#pragma unroll
  for (int p = 0; p < NP; ++p) plane(aout, p, nc)[cell] = ST(phi[p]);
  plane(aout, C::A_FS, nc)[cell] = ST(1.0 - fl);
}

// ---------------------------------------------------------------------------
// Fill: the finite-difference fields of one footprint cell of a real layer
// into the LDS ring (phi_p, f_s from the moments pass, rho by eq. (eq2),
// u^{n-1}).
// ---------------------------------------------------------------------------
template <class C>
__host__ __device__ inline void fill_cell(const StepArgs<typename C::S>& a, const KParams& P,
                                          Smem<C>& sm, const BlockPos& bp, int f, int w) {
  using R = typename C::R;
  using ST = typename C::S;
  constexpr int NP = C::NP;
  const int lx = f % C::LX, ly = f / C::LX;
  int lat = wrapf(bp.tx0 + lx - 1, P.nx);
  if (C::DIM == 3) lat += wrapf(bp.ty0 + ly - 1, P.ny) * P.nx;
  const long long nc = P.ncell;
  const int cell = w * (int)P.area + lat;
  const ST* __restrict__ mom = a.mom;
  const ST* __restrict__ ain = a.ain;
  const int s = slot(w);
  R phi[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    phi[p] = R(plane(mom, p, nc)[cell]);
    sm.phi[s][p][f] = phi[p];
  }
  const R fs = R(plane(mom, C::A_FS, nc)[cell]);
  sm.fs[s][f] = fs;
  sm.rho[s][f] = mixture<R, NP>(phi, fs, P.rho_s, P.rho_l);
#pragma unroll
  for (int d = 0; d < C::DIM; ++d) sm.u[s][d][f] = R(plane(ain, C::A_U + d, nc)[cell]);
}

// Ghost layer beyond a wall-normal face (w = -1 or w = nwn), from the
// boundary layer already in LDS.  At the low face of a wall the order
// parameters follow the geometric wetting rule
//   phi_p(ghost) = phi_p + (4/eps) sum_{q != p} phi_p phi_q cos(theta_pq);
// everything else is copied, except u^{n-1}, which is mirrored at walls
// (zero on the face) and copied at open faces.
template <class C>
__host__ __device__ inline void fill_ghost(const KParams& P, Smem<C>& sm, int f, int w) {
  using R = typename C::R;
  constexpr int NP = C::NP;
  const int face = (w < 0) ? 0 : 1;
  const int sb = slot(face == 0 ? 0 : P.nwn - 1), s = slot(w);
  if (face == 0 && P.flow_bc[0] == BC_WALL) {
    R pb[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) pb[p] = sm.phi[sb][p][f];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      R acc = R(0);
#pragma unroll
      for (int q = 0; q < NP; ++q)
        if (q != p) acc += pb[p] * pb[q] * R(P.cth[p][q]);
      sm.phi[s][p][f] = pb[p] + R(P.four_eps) * acc;
    }
  } else {
#pragma unroll
    for (int p = 0; p < NP; ++p) sm.phi[s][p][f] = sm.phi[sb][p][f];
  }
  sm.fs[s][f] = sm.fs[sb][f];
  sm.rho[s][f] = sm.rho[sb][f];
  const R sgn = (face_flow(P, face) == BC_WALL) ? R(-1) : R(1);
#pragma unroll
  for (int d = 0; d < C::DIM; ++d) sm.u[s][d][f] = sgn * sm.u[sb][d][f];
}

template <class C>
__host__ __device__ inline void fill_layer_cell(const StepArgs<typename C::S>& a, const KParams& P,
                                                Smem<C>& sm, const BlockPos& bp, int f, int w) {
  if (w < 0 || w >= P.nwn)
    fill_ghost<C>(P, sm, f, w);
  else
    fill_cell<C>(a, P, sm, bp, f, w);
}

// Push of one post-collision population: x + c_i inside the domain gets it;
// a link leaving through a wall-normal face (face = 0 or 1, return -1)
// instead stores the face's value for the opposite, incoming direction at
// this cell.  Only the first and last layer (EDGE) have such links; the
// test is uniform across a block.
template <class C, bool EDGE>
__host__ __device__ inline int push_index(const KParams& P, int i, int gx, int gy, int w, int& face) {
  using L = typename C::L;
  const int tw = w + L::cw(i);
  face = -1;
  if (EDGE && (tw < 0 || tw >= P.nwn)) {
    face = tw < 0 ? 0 : 1;
    return -1;
  }
  int lat = wrap1(gx + L::cl0(i), P.nx);
  if (C::DIM == 3) lat += wrap1(gy + L::cl1(i), P.ny) * P.nx;
  return tw * (int)P.area + lat;
}

// c_i . v for direction i of the lattice (components +-1 or 0 folded at
// compile time once the direction loops are unrolled).
template <class C, typename R>
__host__ __device__ inline R cdot(int i, const R* v) {
  using L = typename C::L;
  R s = R(0);
#pragma unroll
  for (int d = 0; d < C::DIM; ++d) {
    if (L::c(i, d) > 0) s += v[d];
    if (L::c(i, d) < 0) s -= v[d];
  }
  return s;
}

// ---------------------------------------------------------------------------
// Process: steps 3-7 of the time step for the interior cell of thread tid in
// layer w.  MOMENTS = true writes one macroscopic field instead of the
// collision; EDGE must be set for the first and last layer.
// ---------------------------------------------------------------------------
template <class C, bool MOMENTS, bool EDGE>
__host__ __device__ inline void process_cell(const StepArgs<typename C::S>& a, const KParams& P,
                                             Smem<C>& sm, const BlockPos& bp, int tid, int w) {
  using R = typename C::R;
  using ST = typename C::S;  // storage type
  using L = typename C::L;
  constexpr int Q = C::Q, NP = C::NP, DIM = C::DIM;
  const int tx = tid % C::TX, ty = tid / C::TX;
  const int gx = bp.tx0 + tx, gy = bp.ty0 + ty;
  if (gx >= P.nx) return;
  if (DIM == 3 && gy >= P.ny) return;
  const long long nc = P.ncell;
  const int lat = (DIM == 3) ? gy * P.nx + gx : gx;
  const int cell = w * (int)P.area + lat;
  const int fc = (DIM == 3) ? (ty + 1) * C::LX + tx + 1 : tx + 1;
  const int s0 = slot(w);
  const ST* __restrict__ pin = a.pin;
  const ST* __restrict__ ain = a.ain;
  ST* __restrict__ pout = a.pout;
  // The flow populations (step 5) are loaded first, so that their latency
  // overlaps the LDS reads and arithmetic of the finite differences.
  R fpop[Q];
  if (!MOMENTS) {
#pragma unroll
    for (int i = 0; i < Q; ++i) fpop[i] = R(plane(pin, i, nc)[cell]);
  }

  // Own moments (identical to the values the neighbours see).
  R phi[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) phi[p] = sm.phi[s0][p][fc];
  const R fs = sm.fs[s0][fc];
  const R rho = sm.rho[s0][fc];
  R psi = R(0);
#pragma unroll
  for (int p = 0; p < NP; ++p)
    if (P.freezes[p]) psi += phi[p];
  R uprev[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) uprev[d] = sm.u[s0][d][fc];

  // Step 3: isotropic central differences at time n,
  // grad X = 3 sum_i w_i c_i X(x+c_i), lap X = 6 sum_i w_i [X(x+c_i) - X(x)].
  R gphi[NP][DIM], lphi[NP], grho[DIM], gfp[NP][DIM], gu[DIM];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    lphi[p] = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) gphi[p][d] = gfp[p][d] = R(0);
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d) grho[d] = gu[d] = R(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int sn = slot(w + L::cw(i));
    const int fn = fc + L::cl0(i) + L::cl1(i) * C::LX;
    const R wi = wgt<R, DIM>(i);
    const R fsn = sm.fs[sn][fn];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const R X = sm.phi[sn][p][fn];
      const R t = wi * X;
      const R tf = wi * (fsn * X);
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        if (L::c(i, d) > 0) {
          gphi[p][d] += t;
          gfp[p][d] += tf;
        }
        if (L::c(i, d) < 0) {
          gphi[p][d] -= t;
          gfp[p][d] -= tf;
        }
      }
      lphi[p] += wi * (X - phi[p]);
    }
    const R tr = wi * sm.rho[sn][fn];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const R tu = wi * sm.u[sn][d][fn];
      if (L::c(i, d) > 0) {
        grho[d] += tr;
        gu[d] += tu;
      }
      if (L::c(i, d) < 0) {
        grho[d] -= tr;
        gu[d] -= tu;
      }
    }
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    lphi[p] *= R(6);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      gphi[p][d] *= R(3);
      gfp[p][d] *= R(3);
    }
  }
  R Ddiv = R(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    grho[d] *= R(3);
    Ddiv += R(3) * gu[d];
  }

  // Step 4: interface physics of Sec. 2.  Pairwise normals via the quotient
  // rule, v = phi_q grad phi_p - phi_p grad phi_q, |v| regularised by 1e-12;
  // each pair adds 4 phi_p phi_q / eps n_pq to R_p and its negative to R_q.
  R Rp[NP][DIM], mup[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int d = 0; d < DIM; ++d) Rp[p][d] = R(0);
  const R ieps = R(1) / R(P.eps);
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int q = p + 1; q < NP; ++q) {
      R v[DIM], vv = R(0);
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        v[d] = phi[q] * gphi[p][d] - phi[p] * gphi[q][d];
        vv += v[d] * v[d];
      }
      const R sc = R(4) * phi[p] * phi[q] * ieps / sqrt(vv + R(1e-24));
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        Rp[p][d] += sc * v[d];
        Rp[q][d] -= sc * v[d];
      }
    }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    R bulk = R(0), gterm = R(0);
    const R gp = gprime(phi[p]);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      if (q == p) continue;
      bulk += R(2) * R(P.beta[p][q]) * (gp - gprime(phi[p] + phi[q]));
      gterm += R(P.kpq[p][q]) * lphi[q];
    }
    mup[p] = bulk - gterm;
  }
  R F[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    R fsd = R(0);
#pragma unroll
    for (int p = 0; p < NP; ++p) fsd += mup[p] * gphi[p][d];
    F[d] = fsd + rho * R(P.grav[d]);
  }

  // Step 5: flow macros (the moments mode loads the flow populations here).
  if (MOMENTS) {
#pragma unroll
    for (int i = 0; i < Q; ++i) fpop[i] = R(plane(pin, i, nc)[cell]);
  }
  R mom[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) mom[d] = R(0);
#pragma unroll
  for (int i = 1; i < Q; ++i)
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (L::c(i, d) > 0) mom[d] += fpop[i];
      if (L::c(i, d) < 0) mom[d] -= fpop[i];
    }
  const R irho = R(1) / rho;
  const R ws = fs * psi;
  R u[DIM], Fa[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const R us = (mom[d] + R(0.5) * F[d]) * irho;
    const R acc = ws * (R(0) - us);
    u[d] = us + R(0.5) * acc;
    Fa[d] = F[d] + rho * acc;  // F + rho a
  }
  // mdot = -(1/rho) sum_{p freezing} (rho_p^s - rho_p^l) D(f_s phi_p)/Dt
  R msum = R(0);
  const R fsp = R(plane(ain, C::A_FS, nc)[cell]);
  R phip[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) phip[p] = R(plane(ain, p, nc)[cell]);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    if (!P.freezes[p]) continue;
    R ug = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) ug += u[d] * gfp[p][d];
    msum += R(P.rho_s[p] - P.rho_l[p]) * (fs * phi[p] - fsp * phip[p] + ug);
  }
  const R mdot = -msum * irho;
  R ugr = R(0), uu = R(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    ugr += u[d] * grho[d];
    uu += u[d] * u[d];
  }
  const R S = rho * mdot + ugr;
  // Forcing F_i = w_i [S + 3 c.(F + rho a) + 9/2 (c c - I/3) : Lambda],
  // Lambda = u F + F u + (2/d) rho cs2 S I; (c c - I/3):Lambda =
  // 2 (c.u)(c.F) + (2/d) rho cs2 S (|c|^2 - d/3) - 2/3 u.F.
  R uF = R(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) uF += u[d] * F[d];
  const R lam_iso = R(2.0 / DIM) * rho * R(1.0 / 3.0) * S;
  const R mu = mixture<R, NP>(phi, fs, P.mu_s, P.mu_l);
  const R tau_f = R(3) * mu * irho + R(0.5);
  const R itf = R(1) / tau_f;
  const R sfac = R(1) - R(0.5) * itf;
  const R w0 = wgt<R, DIM>(0);
  R sf = R(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) sf += fpop[i];
  // F_0 (c_0 = 0): w_0 [S + 9/2 (-1/3) tr Lambda]
  const R F0 = w0 * (S + R(4.5) * (-R(2.0 / 3.0) * uF - R(DIM) * R(1.0 / 3.0) * lam_iso));
  const R s0u = w0 * (-R(1.5) * uu);
  const R pr = R(1.0 / 3.0) / (R(1) - w0) * (sf + R(0.5) * S + (tau_f - R(0.5)) * F0 + rho * s0u);

  const int lh = NP + 1;
  if (MOMENTS) {
    R hpop[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) hpop[i] = R(plane(pin, lh * Q + i, nc)[cell]);
    double Td, fl;
    const double rhoH = own_enthalpy<C>(P, phi, hpop, R(plane(ain, C::A_Q, nc)[cell]), Td, fl);
    const int k = a.mfield;
    double v = 0.0;
    if (k < NP) v = double(phi[k]);
    else if (k == NP) v = rhoH;
    else if (k == NP + 1) v = Td;
    else if (k == NP + 2) v = fl;
    else if (k == NP + 3) v = double(rho);
    else if (k < NP + 4 + DIM) v = double(u[k - NP - 4]);
    else if (k == NP + 4 + DIM) v = double(pr);
    else v = double(mdot);
    a.mout[cell] = v;
    return;
  }

  // Step 6-7: collisions and push streaming.
  // Flow LB: f^eq_0 = 3p (w_0 - 1) + rho s_0, f^eq_i = 3p w_i + rho s_i.
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R cu = cdot<C>(i, u);
    const R cF = cdot<C>(i, Fa);
    const R cFs = cdot<C>(i, F);
    const R wi = wgt<R, DIM>(i);
    const R c2 = R(L::c(i, 0) * L::c(i, 0) + L::c(i, 1) * L::c(i, 1) + L::c(i, 2) * L::c(i, 2));
    const R qq = R(2) * cu * cFs - R(2.0 / 3.0) * uF + lam_iso * (c2 - R(DIM) * R(1.0 / 3.0));
    const R Fi = wi * (S + R(3) * cF + R(4.5) * qq);
    const R si = wi * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
    const R fe = (i == 0) ? R(3) * pr * (w0 - R(1)) + rho * si : R(3) * pr * wi + rho * si;
    const R post = fpop[i] - (fpop[i] - fe) * itf + sfac * Fi;
    int face;
    const int t = push_index<C, EDGE>(P, i, gx, gy, w, face);
    if (!EDGE || t >= 0) {
      plane(pout, i, nc)[t] = ST(post);
    } else {
      const int ib = L::opp(i);
      R val;
      if (face_flow(P, face) == BC_WALL) {
        val = post;  // halfway bounce-back
      } else {
        // open face: ghost at pressure 0 with this cell's u and rho
        const R cub = -cu;
        const R wb = wgt<R, DIM>(ib);
        const R sb = wb * (R(3) * cub + R(4.5) * cub * cub - R(1.5) * uu);
        const R feb = R(3) * pr * wb + rho * sb;
        val = rho * sb + (R(1) - itf) * (fpop[ib] - feb);
      }
      plane(pout, ib, nc)[cell] = ST(val);
    }
  }

  // Phase-field LBs: g^eq = w_i phi (1 + 3 c.u),
  // G = w_i [3 c.(phi u - phi^{n-1} u^{n-1}) + c.R_p] + w_i phi D.
  const R itg = R(1) / R(P.tau_g);
  const R gfac = R(1) - R(0.5) * itg;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    R dpu[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) dpu[d] = R(3) * (phi[p] * u[d] - phip[p] * uprev[d]) + Rp[p][d];
    const int l = 1 + p;
    R gpop[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) gpop[i] = R(plane(pin, l * Q + i, nc)[cell]);
    const R phD = phi[p] * Ddiv;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R cu = cdot<C>(i, u);
      const R wi = wgt<R, DIM>(i);
      const R Gi = wi * (cdot<C>(i, dpu) + phD);
      const R ge = wi * phi[p] * (R(1) + R(3) * cu);
      const R post = gpop[i] - (gpop[i] - ge) * itg + gfac * Gi;
      int face;
      const int t = push_index<C, EDGE>(P, i, gx, gy, w, face);
      if (!EDGE || t >= 0) {
        plane(pout, l * Q + i, nc)[t] = ST(post);
      } else {
        const int ib = L::opp(i);
        R val;
        if (face_flow(P, face) == BC_WALL) {
          val = post;
        } else {
          const R geb = wgt<R, DIM>(ib) * phi[p] * (R(1) - R(3) * cu);
          val = geb + (R(1) - itg) * (gpop[ib] - geb);
        }
        plane(pout, l * Q + ib, nc)[cell] = ST(val);
      }
    }
  }

  // Own rho H (float64) and T, eq. (H), from the h populations.
  R hpop[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) hpop[i] = R(plane(pin, lh * Q + i, nc)[cell]);
  double Td, fl;
  const double rhoH = own_enthalpy<C>(P, phi, hpop, R(plane(ain, C::A_Q, nc)[cell]), Td, fl);
  const R T = R(Td);

  // Total-enthalpy LB: h^eq_0 = rhoH - E_ref T + w_0 (E_ref T - 3/2 rho C_p T u.u),
  // h^eq_i = w_i [E_ref T + rho C_p T (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)],
  // H_i = w_i rho C_p T D, tau_h = 3 lambda / E_ref + 1/2.  The rest
  // population is updated in float64 (it carries the latent heat offset).
  const R lam = mixture<R, NP>(phi, fs, P.lam_s, P.lam_l);
  const R cp = mixture<R, NP>(phi, fs, P.cp_s, P.cp_l);
  const R rhocp = rho * cp;
  const R Eref = R(P.E_ref);
  const R tau_h = R(3) * lam / Eref + R(0.5);
  const R ith = R(1) / tau_h;
  const R hfac = R(1) - R(0.5) * ith;
  const R ET = Eref * T, CT = rhocp * T, HD = CT * Ddiv;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R wi = wgt<R, DIM>(i);
    const R cu = cdot<C>(i, u);
    R post;
    if (i == 0) {
      const double Er = P.E_ref;
      const double rc = double(rhocp);
      const double he0 = rhoH - Er * Td + double(w0) * (Er * Td - 1.5 * rc * Td * double(uu));
      const double H0 = double(wi) * rc * Td * double(Ddiv);
      const double ithd = double(ith);
      const double h0 = double(hpop[0]);
      post = R(h0 - (h0 - he0) * ithd + (1.0 - 0.5 * ithd) * H0);
    } else {
      const R he = wi * (ET + CT * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
      post = hpop[i] - (hpop[i] - he) * ith + hfac * (wi * HD);
    }
    int face;
    const int t = push_index<C, EDGE>(P, i, gx, gy, w, face);
    if (!EDGE || t >= 0) {
      plane(pout, lh * Q + i, nc)[t] = ST(post);
    } else {
      const int ib = L::opp(i);
      R val;
      if (face_flow(P, face) == BC_WALL && face_therm(P, face) == TBC_ADIABATIC) {
        val = post;
      } else {
        // Ghost node half a cell outside the face at T_g (Dirichlet:
        // 2 T_face - T), velocity 0 at walls and u at open faces; this
        // cell's non-equilibrium part.
        const R Tg = (face_therm(P, face) == TBC_DIRICHLET) ? R(2) * R(face_T(P, face)) - T : T;
        const bool open = face_flow(P, face) == BC_OPEN;
        const R cub = open ? -cu : R(0);
        const R ugug = open ? uu : R(0);
        const R wb = wgt<R, DIM>(ib);
        const R hg = wb * (Eref * Tg + rhocp * Tg * (R(3) * cub + R(4.5) * cub * cub - R(1.5) * ugug));
        const R heb = wb * (ET + CT * (-R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
        val = hg + (R(1) - ith) * (hpop[ib] - heb);
      }
      plane(pout, lh * Q + ib, nc)[cell] = ST(val);
    }
  }

  // Lagged fields for the next step (phi_p and f_s were written by the
  // moments pass).
  ST* __restrict__ aout = a.aout;
#pragma unroll
  for (int d = 0; d < DIM; ++d) plane(aout, C::A_U + d, nc)[cell] = ST(u[d]);
  plane(aout, C::A_DIV, nc)[cell] = ST(Ddiv);
  plane(aout, C::A_Q, nc)[cell] = ST(HD);
}

}  // namespace lbf
