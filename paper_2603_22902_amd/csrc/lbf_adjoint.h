// Discrete adjoint (reverse mode) of one coupled-LB time step of
// arXiv:2603.22902, Sec. 3, written by hand from the forward step in
// lbf_step.h, for gradients of an objective of the final state with respect
// to the wall temperatures, the latent heats and the wetting cosines.
//
// With x^{n+1} = S(x^n, theta), the reverse step maps the adjoint of the
// state after the step, lambda^{n+1}, to the adjoint of the state before it,
//   lambda^n = (dS/dx^n)^T lambda^{n+1},
// and adds lambda^{n+1} . dS/dtheta to the parameter gradient.  The state is
// the populations (f, g_p, h) and the lagged fields (phi_p, f_s, u, D, q), in
// the forward layout; the adjoint buffers use the same layout, except that
// the adjoint of the lagged fields carries N + 1 more planes: the moments
// reverse adds one value per cell to every g_{i,p} (phi_p's adjoint over
// 1 - D/2) and to every h_i (rho H's adjoint).  These stay as the per-cell
// scalars A_GS + p and A_GS + N, and every reader of a population adjoint
// adds them (adj_pop), instead of a read-modify-write of all (N+1) Q values.
//
// A reverse step is three passes over the cells (one thread per cell):
//   1. adj_moment_cell   the forward moments phi_p, f_s, rho H of x^n
//                        (recomputed from the stored state; skipped when
//                        x^{n+1} is at hand, whose first N + 1 lagged planes
//                        are phi_p^n, f_s^n, with rho H then written by
//                        pass 2);
//   2. adj_collide_cell  the transpose of the push (each cell pulls the
//                        adjoints of the values it wrote, including the
//                        face links), then the reverse of the collisions,
//                        flow macros, volume source, interface terms and
//                        the own-cell enthalpy inversion.  It writes the
//                        adjoints of its pre-collision populations, of its
//                        finite-difference outputs (grad phi_p, lap phi_p,
//                        grad rho, grad f_s phi_p, div u^{n-1}), of its own
//                        phi_p, f_s and of its lagged inputs;
//   3. adj_gather_cell   the transpose of the finite differences (each cell
//                        gathers from the cells that read it, including the
//                        wetting ghost layer), of the mixture density and of
//                        the moments and the enthalpy inversion.
// The inversion and the regularised norm are piecewise smooth: the reverse
// takes the derivative of the branch the forward step took.
//
// Every function is __host__ __device__ so that the host emulator runs the
// same code for the CPU checks against finite differences.
#pragma once

#include <type_traits>

#include "lbf_step.h"

namespace lbf {

// Parameter-gradient slots: T_face[2], latent[MAXP], cth[MAXP][MAXP].
constexpr int PAR_TFACE = 0, PAR_LATENT = 2, PAR_CTH = 2 + MAXP;
constexpr int NPAR = 2 + MAXP + MAXP * MAXP;

// Work planes of the reverse step (arithmetic type R, one value per cell).
template <class C>
struct AdjLayout {
  static constexpr int N = C::NP, D = C::DIM;
  // forward moments of x^n
  static constexpr int M_PHI = 0, M_FS = N, M_RHOH = N + 1, NMOM = N + 2;
  // adjoints of the finite-difference outputs of each cell
  static constexpr int F_GPHI = NMOM;                    // [p*D + d]
  static constexpr int F_LPHI = F_GPHI + N * D;          // [p]
  static constexpr int F_GRHO = F_LPHI + N;              // [d]
  static constexpr int F_GFP = F_GRHO + D;               // [p*D + d]
  static constexpr int F_DIV = F_GFP + N * D;
  // adjoints of the own phi_p, f_s (as the collision read them)
  static constexpr int O_PHI = F_DIV + 1, O_FS = O_PHI + N;
  // adjoints of the lagged inputs read by the collision of each cell
  static constexpr int L_PHI = O_FS + 1, L_FS = L_PHI + N, L_U = L_FS + 1, L_Q = L_U + D;
  static constexpr int NWORK = L_Q + 1;
};

template <class C>
struct AdjArgs {
  using S = typename C::S;
  using R = typename C::R;
  const S* pin;   // forward state x^n: populations
  const S* ain;   //                    lagged fields
  const S* lpin;  // adjoint of x^{n+1}
  const S* lain;
  S* lpout;       // adjoint of x^n
  S* laout;
  R* work;        // AdjLayout planes
  const S* mom;   // lagged fields of x^{n+1} (phi_p^n, f_s^n), or NULL: the
                  // moment planes of work
};

template <class C>
__host__ __device__ inline typename C::R* wplane(const AdjArgs<C>& a, int k, long long nc) {
  return a.work + (long long)k * nc;
}

// A buffer of nplanes planes of nc values, read and written through a
// buffer resource on the device: the start and size sit in scalar
// registers, and an access takes the plane's byte offset (the same for the
// whole wave, in a scalar register) and the cell's (32-bit, per lane).
// The hardware checks the range: outside the buffer a read gives 0 and a
// write is dropped.  Against 64-bit per-lane addresses this frees the
// registers of one address pair per access in flight.  The host (the
// emulator) indexes the pointer.  Spans must stay below 2 GiB (checked with
// the adjoint's layout).
template <typename T>
struct GBuf {
  T* p;
  int nc, bytes;
  __host__ __device__ GBuf(T* ptr, long long ncell, int nplanes)
      : p(ptr), nc((int)ncell), bytes((int)(ncell * nplanes * (long long)sizeof(T))) {}
#if defined(__HIP_DEVICE_COMPILE__)
  __device__ __amdgpu_buffer_rsrc_t rsrc() const {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(static_cast<const void*>(p)), 0, bytes, 0x00020000);
  }
#endif
  __host__ __device__ typename std::remove_const<T>::type ld(int k, int i) const {
    using U = typename std::remove_const<T>::type;
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(U) == 4)
      return __builtin_bit_cast(U, __builtin_amdgcn_raw_buffer_load_b32(rsrc(), i * 4, k * nc * 4, 0));
    else
      return __builtin_bit_cast(U, __builtin_amdgcn_raw_buffer_load_b64(rsrc(), i * 8, k * nc * 8, 0));  // 2 dwords
#else
    return p[(long long)k * nc + i];
#endif
  }
  __host__ __device__ void st(int k, int i, T v) const {
#if defined(__HIP_DEVICE_COMPILE__)
    using V2 = unsigned __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rsrc(), i * 4, k * nc * 4, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), rsrc(), i * 8, k * nc * 8, 0);
#else
    p[(long long)k * nc + i] = v;
#endif
  }
};

// Planes of the per-cell population scalars in the adjoint of the lagged
// fields (after the N + DIM + 3 planes of the forward layout).
template <class C>
struct AdjScal {
  static constexpr int GS = C::NAUX, HS = C::NAUX + C::NP, NLA = C::NAUX + C::NP + 1;
};

// Adjoint of population i of lattice l at a cell: the stored value plus the
// cell's scalar of that lattice (none for f).
template <class C>
__host__ __device__ inline typename C::R adj_pop(const typename C::S* lp, const typename C::S* la, int l, int i,
                                                 int cell, long long nc) {
  using R = typename C::R;
  R v = R(plane(lp, l * C::Q + i, nc)[cell]);
  if (l >= 1) v += R(plane(la, AdjScal<C>::GS + l - 1, nc)[cell]);
  return v;
}

// phi_p and f_s of x^n at a cell.
template <class C>
__host__ __device__ inline typename C::R m_phi(const AdjArgs<C>& a, int p, int cell, long long nc) {
  using R = typename C::R;
  return a.mom ? R(plane(a.mom, p, nc)[cell]) : wplane(a, AdjLayout<C>::M_PHI + p, nc)[cell];
}
template <class C>
__host__ __device__ inline typename C::R m_fs(const AdjArgs<C>& a, int cell, long long nc) {
  using R = typename C::R;
  return a.mom ? R(plane(a.mom, C::A_FS, nc)[cell]) : wplane(a, AdjLayout<C>::M_FS, nc)[cell];
}

__host__ __device__ inline double gsecond(double x) { return 2.0 - 12.0 * x + 12.0 * x * x; }
__host__ __device__ inline float gsecond(float x) { return 2.0f - 12.0f * x + 12.0f * x * x; }

// Derivatives of eq. (H) as evaluated by invert() at (phi, rho H), for the
// branch taken: dT/d(rho H), dT/dphi_p, dT/dL_p, and the same for f_l.
template <int NP, typename R>
__host__ __device__ inline void invert_grad(const KParams& P, const R* phi, double rhoH, double& dT_dH,
                                            double* dT_dphi, double* dT_dL, double& dfl_dH,
                                            double* dfl_dphi, double* dfl_dL) {
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
  dT_dH = dfl_dH = 0.0;
#pragma unroll
  for (int p = 0; p < NP; ++p) dT_dphi[p] = dT_dL[p] = dfl_dphi[p] = dfl_dL[p] = 0.0;
  if (rhoH < Es) {
    const double a = rs * cs;
    dT_dH = 1.0 / a;
#pragma unroll
    for (int p = 0; p < NP; ++p) dT_dphi[p] = -rhoH / (a * a) * (P.rho_s[p] * cs + rs * P.cp_s[p]);
  } else if (rhoH > El) {
    const double a = rl * cl;
    dT_dH = 1.0 / a;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const double da = P.rho_l[p] * cl + rl * P.cp_l[p];
      const double dEl = da * Tm + P.rho_l[p] * P.latent[p];
      dT_dphi[p] = -dEl / a - (rhoH - El) / (a * a) * da;
      dT_dL[p] = -double(phi[p]) * P.rho_l[p] / a;
    }
  } else if (El > Es) {
    const double dE = El - Es;
    const double fl = (rhoH - Es) / dE;
    dfl_dH = 1.0 / dE;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const double dEs = (P.rho_s[p] * cs + rs * P.cp_s[p]) * Tm;
      const double dEl = (P.rho_l[p] * cl + rl * P.cp_l[p]) * Tm + P.rho_l[p] * P.latent[p];
      dfl_dphi[p] = (fl - 1.0) / dE * dEs - fl / dE * dEl;
      dfl_dL[p] = -fl / dE * double(phi[p]) * P.rho_l[p];
    }
  }
}

// Adjoint of the mixture law (eq. (eq2)): xb -> phib, fsb.
template <typename R, int NP>
__host__ __device__ inline void mixture_adj(R xb, const R* phi, R fs, const double* xs, const double* xl,
                                            R* phib, R& fsb) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    phib[p] += xb * (fs * R(xs[p]) + (R(1) - fs) * R(xl[p]));
    fsb += xb * phi[p] * (R(xs[p]) - R(xl[p]));
  }
}

// ---------------------------------------------------------------------------
// Pass 1: forward moments of x^n (the moments pass plus rho H).
// ---------------------------------------------------------------------------
template <class C>
__host__ __device__ inline void adj_moment_cell(const AdjArgs<C>& a, const KParams& P, int cell) {
  using R = typename C::R;
  using L = AdjLayout<C>;
  constexpr int Q = C::Q, NP = C::NP;
  const long long nc = P.ncell;
  // as the forward moments pass (compensated sums, float64 division)
  const double div = double(plane(a.ain, C::A_DIV, nc)[cell]);
  const double qv = double(plane(a.ain, C::A_Q, nc)[cell]);
  const double idiv = 1.0 / (1.0 - 0.5 * div);
  double phid[NP];
  R phi[NP];
  for (int p = 0; p < NP; ++p) {
    MomSum<typename C::S> sum;
    for (int i = 0; i < Q; ++i) sum.add(plane(a.pin, (1 + p) * Q + i, nc)[cell]);
    phid[p] = double(typename C::S(sum.value() * idiv));
    phi[p] = R(phid[p]);
  }
  double sh = 0.0;
  for (int i = 0; i < Q; ++i) sh += double(plane(a.pin, (NP + 1) * Q + i, nc)[cell]);
  const double rhoH = sh + 0.5 * qv;
  double T, fl;
  invert<NP>(P, phid, rhoH, T, fl);
  for (int p = 0; p < NP; ++p) wplane(a, L::M_PHI + p, nc)[cell] = phi[p];
  wplane(a, L::M_FS, nc)[cell] = R(typename C::S(1.0 - fl));
  wplane(a, L::M_RHOH, nc)[cell] = R(rhoH);
}

// Finite-difference inputs of the neighbour of cell (gx, gy, layer w) in
// direction i, as the forward fill and ghost rules give them: phi_p and f_s
// of the moments, rho by the mixture law, u^{n-1}; beyond a wall-normal
// face the ghost copies the boundary cell (wetting rule for phi at a low
// wall, u mirrored at walls).  base is the cell the value derives from.
template <class C>
__host__ __device__ inline void nb_fields(const AdjArgs<C>& a, const KParams& P, int gx, int gy, int w,
                                          int i, typename C::R* phi, typename C::R& fs,
                                          typename C::R& rho, typename C::R* up) {
  using R = typename C::R;
  using Lt = typename C::L;
  constexpr int NP = C::NP;
  const long long nc = P.ncell;
  int lat = wrap1(gx + Lt::cl0(i), P.nx);
  if (C::DIM == 3) lat += wrap1(gy + Lt::cl1(i), P.ny) * P.nx;
  const int tw = w + Lt::cw(i);
  const bool ghost = tw < 0 || tw >= P.nwn;
  const int face = tw < 0 ? 0 : 1;
  const int bw = ghost ? (face == 0 ? 0 : P.nwn - 1) : tw;
  const int b = bw * (int)P.area + lat;
  R pb[NP];
  for (int p = 0; p < NP; ++p) pb[p] = m_phi<C>(a, p, b, nc);
  fs = m_fs<C>(a, b, nc);
  rho = mixture<R, NP>(pb, fs, P.rho_s, P.rho_l);
  const R sgn = (ghost && face_flow(P, face) == BC_WALL) ? R(-1) : R(1);
  for (int d = 0; d < C::DIM; ++d) up[d] = sgn * R(plane(a.ain, C::A_U + d, nc)[b]);
  if (ghost && face == 0 && P.flow_bc[0] == BC_WALL) {
    for (int p = 0; p < NP; ++p) {
      R acc = R(0);
      for (int q = 0; q < NP; ++q)
        if (q != p) acc += pb[p] * pb[q] * R(P.cth[p][q]);
      phi[p] = pb[p] + R(P.four_eps) * acc;
    }
  } else {
    for (int p = 0; p < NP; ++p) phi[p] = pb[p];
  }
}

// ---------------------------------------------------------------------------
// Pass 2: reverse of the collide pass for one cell.  gpar accumulates the
// cell's parameter-gradient contributions (NPAR doubles).
// ---------------------------------------------------------------------------
// The neighbour fields of the forward recompute read from global memory
// (nb_fields); a tiled kernel reads them from its LDS ring instead.
template <class C>
struct NbGlobal {
  const AdjArgs<C>* a;
  int gx, gy, w;
  __host__ __device__ void operator()(const KParams& P, int i, typename C::R* phi, typename C::R& fs,
                                      typename C::R& rho, typename C::R* up) const {
    nb_fields<C>(*a, P, gx, gy, w, i, phi, fs, rho, up);
  }
};

template <class C, class NB>
__host__ __device__ inline void adj_collide_cell(const AdjArgs<C>& a, const KParams& P, int cell, double* gpar,
                                                 const NB& nb) {
  using R = typename C::R;
  using ST = typename C::S;
  using Lt = typename C::L;
  using L = AdjLayout<C>;
  constexpr int Q = C::Q, NP = C::NP, DIM = C::DIM;
  const long long nc = P.ncell;
  const int area = (int)P.area;
  const int w = cell / area, lat = cell - w * area;
  const int gx = lat % P.nx, gy = lat / P.nx;
  const ST* pin = a.pin;
  const ST* ain = a.ain;
  const GBuf<const ST> bpi(pin, nc, (NP + 2) * Q), bai(ain, nc, C::NAUX);

  // ---- forward recompute (as process_cell) ----
  R phi[NP];
  for (int p = 0; p < NP; ++p) phi[p] = m_phi<C>(a, p, cell, nc);
  const R fs = m_fs<C>(a, cell, nc);
  const R rho = mixture<R, NP>(phi, fs, P.rho_s, P.rho_l);
  R psi = R(0);
  for (int p = 0; p < NP; ++p)
    if (P.freezes[p]) psi += phi[p];
  R uprev[DIM];
  for (int d = 0; d < DIM; ++d) uprev[d] = R(bai.ld(C::A_U + d, cell));

  R gphi[NP][DIM], lphi[NP], grho[DIM], gfp[NP][DIM], gu[DIM];
  for (int p = 0; p < NP; ++p) {
    lphi[p] = R(0);
    for (int d = 0; d < DIM; ++d) gphi[p][d] = gfp[p][d] = R(0);
  }
  for (int d = 0; d < DIM; ++d) grho[d] = gu[d] = R(0);
  for (int i = 1; i < Q; ++i) {
    R X[NP], fsn, rn, un[DIM];
    nb(P, i, X, fsn, rn, un);
    const R wi = wgt<R, DIM>(i);
    for (int p = 0; p < NP; ++p) {
      const R t = wi * X[p];
      const R tf = wi * (fsn * X[p]);
      for (int d = 0; d < DIM; ++d) {
        if (Lt::c(i, d) > 0) {
          gphi[p][d] += t;
          gfp[p][d] += tf;
        }
        if (Lt::c(i, d) < 0) {
          gphi[p][d] -= t;
          gfp[p][d] -= tf;
        }
      }
      lphi[p] += wi * (X[p] - phi[p]);
    }
    const R tr = wi * rn;
    for (int d = 0; d < DIM; ++d) {
      const R tu = wi * un[d];
      if (Lt::c(i, d) > 0) {
        grho[d] += tr;
        gu[d] += tu;
      }
      if (Lt::c(i, d) < 0) {
        grho[d] -= tr;
        gu[d] -= tu;
      }
    }
  }
  for (int p = 0; p < NP; ++p) {
    lphi[p] *= R(6);
    for (int d = 0; d < DIM; ++d) {
      gphi[p][d] *= R(3);
      gfp[p][d] *= R(3);
    }
  }
  R Ddiv = R(0);
  for (int d = 0; d < DIM; ++d) {
    grho[d] *= R(3);
    Ddiv += R(3) * gu[d];
  }
  const R ieps = R(1) / R(P.eps);
  R Rp[NP][DIM];
  for (int p = 0; p < NP; ++p)
    for (int d = 0; d < DIM; ++d) Rp[p][d] = R(0);
  for (int p = 0; p < NP; ++p)
    for (int q = p + 1; q < NP; ++q) {
      R v[DIM], vv = R(0);
      for (int d = 0; d < DIM; ++d) {
        v[d] = phi[q] * gphi[p][d] - phi[p] * gphi[q][d];
        vv += v[d] * v[d];
      }
      const R sc = R(4) * phi[p] * phi[q] * ieps / sqrt(vv + R(1e-24));
      for (int d = 0; d < DIM; ++d) {
        Rp[p][d] += sc * v[d];
        Rp[q][d] -= sc * v[d];
      }
    }
  R mup[NP];
  for (int p = 0; p < NP; ++p) {
    R bulk = R(0), gterm = R(0);
    const R gp = gprime(phi[p]);
    for (int q = 0; q < NP; ++q) {
      if (q == p) continue;
      bulk += R(2) * R(P.beta[p][q]) * (gp - gprime(phi[p] + phi[q]));
      gterm += R(P.kpq[p][q]) * lphi[q];
    }
    mup[p] = bulk - gterm;
  }
  R F[DIM];
  for (int d = 0; d < DIM; ++d) {
    R fsd = R(0);
    for (int p = 0; p < NP; ++p) fsd += mup[p] * gphi[p][d];
    F[d] = fsd + rho * R(P.grav[d]);
  }
  R fpop[Q];
  for (int i = 0; i < Q; ++i) fpop[i] = R(bpi.ld(i, cell));
  R mom[DIM];
  for (int d = 0; d < DIM; ++d) mom[d] = R(0);
  for (int i = 1; i < Q; ++i)
    for (int d = 0; d < DIM; ++d) {
      if (Lt::c(i, d) > 0) mom[d] += fpop[i];
      if (Lt::c(i, d) < 0) mom[d] -= fpop[i];
    }
  const R irho = R(1) / rho;
  const R ws = fs * psi;
  R us[DIM], u[DIM], Fa[DIM];
  for (int d = 0; d < DIM; ++d) {
    us[d] = (mom[d] + R(0.5) * F[d]) * irho;
    const R acc = ws * (R(0) - us[d]);
    u[d] = us[d] + R(0.5) * acc;
    Fa[d] = F[d] + rho * acc;
  }
  const R fsp = R(bai.ld(C::A_FS, cell));
  R phip[NP];
  for (int p = 0; p < NP; ++p) phip[p] = R(bai.ld(p, cell));
  R msum = R(0);
  for (int p = 0; p < NP; ++p) {
    if (!P.freezes[p]) continue;
    R ug = R(0);
    for (int d = 0; d < DIM; ++d) ug += u[d] * gfp[p][d];
    msum += R(P.rho_s[p] - P.rho_l[p]) * (fs * phi[p] - fsp * phip[p] + ug);
  }
  const R mdot = -msum * irho;
  R ugr = R(0), uu = R(0), uF = R(0);
  for (int d = 0; d < DIM; ++d) {
    ugr += u[d] * grho[d];
    uu += u[d] * u[d];
    uF += u[d] * F[d];
  }
  const R S = rho * mdot + ugr;
  const R lam_iso = R(2.0 / DIM) * rho * R(1.0 / 3.0) * S;
  const R mu = mixture<R, NP>(phi, fs, P.mu_s, P.mu_l);
  const R tau_f = R(3) * mu * irho + R(0.5);
  const R itf = R(1) / tau_f;
  const R sfac = R(1) - R(0.5) * itf;
  const R w0 = wgt<R, DIM>(0);
  R sf = R(0);
  for (int i = 1; i < Q; ++i) sf += fpop[i];
  const R F0 = w0 * (S + R(4.5) * (-R(2.0 / 3.0) * uF - R(DIM) * R(1.0 / 3.0) * lam_iso));
  const R s0u = w0 * (-R(1.5) * uu);
  const R KP = R(1.0 / 3.0) / (R(1) - w0);
  const R pr = KP * (sf + R(0.5) * S + (tau_f - R(0.5)) * F0 + rho * s0u);
  const R itg = R(1) / R(P.tau_g);
  const R gfac = R(1) - R(0.5) * itg;
  const int lh = NP + 1;
  R hpop[Q];
  for (int i = 0; i < Q; ++i) hpop[i] = R(bpi.ld(lh * Q + i, cell));
  double Td, fl;
  const double rhoH = own_enthalpy<C>(P, phi, hpop, R(bai.ld(C::A_Q, cell)), Td, fl);
  const R T = R(Td);
  const R lam = mixture<R, NP>(phi, fs, P.lam_s, P.lam_l);
  const R cp = mixture<R, NP>(phi, fs, P.cp_s, P.cp_l);
  const R rhocp = rho * cp;
  const R Eref = R(P.E_ref);
  const R tau_h = R(3) * lam / Eref + R(0.5);
  const R ith = R(1) / tau_h;
  const R hfac = R(1) - R(0.5) * ith;
  const R ET = Eref * T, CT = rhocp * T, HD = CT * Ddiv;

  // ---- reverse ----
  R phib[NP], ub[DIM], Fb[DIM], Fab[DIM], Rpb[NP][DIM], phipb[NP], upb[DIM];
  for (int p = 0; p < NP; ++p) {
    phib[p] = phipb[p] = R(0);
    for (int d = 0; d < DIM; ++d) Rpb[p][d] = R(0);
  }
  for (int d = 0; d < DIM; ++d) ub[d] = Fb[d] = Fab[d] = upb[d] = R(0);
  R fsb = R(0), rhob = R(0), uub = R(0), Ddivb = R(0), Sb = R(0), uFb = R(0), lamb = R(0);
  R prb = R(0), itfb = R(0), fspb = R(0), qpb = R(0);
  const ST* lpin = a.lpin;
  const ST* lain = a.lain;
  ST* lpout = a.lpout;

  const GBuf<const ST> blp(lpin, nc, (NP + 2) * Q), bla(lain, nc, AdjScal<C>::NLA);
  const GBuf<ST> blo(lpout, nc, (NP + 2) * Q);
  const GBuf<R> bw(a.work, nc, L::NWORK);

  // adjoints of the lagged fields this cell wrote (u, D, q)
  for (int d = 0; d < DIM; ++d) ub[d] += R(bla.ld(C::A_U + d, cell));
  Ddivb += R(bla.ld(C::A_DIV, cell));
  R HDb = R(bla.ld(C::A_Q, cell));

  // Adjoint of the value written for direction i: at x + c_i for an inner
  // link, or (face link) the opposite direction at this cell.  Both are
  // addressed from the lower of the two planes, whose offset is then the
  // same for the whole wave.
  auto out_adj = [&](int lattice, int i, int& face) -> R {
    int f2;
    const int t = push_index<C, true>(P, i, gx, gy, w, f2);
    face = f2;
    const int ib = Lt::opp(i), k0 = i < ib ? i : ib;
    const int idx = t >= 0 ? t + (i - k0) * (int)nc : cell + (ib - k0) * (int)nc;
    R v = R(blp.ld(lattice * Q + k0, idx));
    if (lattice >= 1) v += R(bla.ld(AdjScal<C>::GS + lattice - 1, t >= 0 ? t : cell));
    return v;
  };

  // Each lattice's Q output adjoints are loaded together before its loop,
  // and every direction runs the same code (no test for a zero adjoint), so
  // the loads issue as one batch.
  R abv[Q];
  int facev[Q];

  // -- enthalpy LB and its face rules --
  R hb[Q];
  for (int i = 0; i < Q; ++i) hb[i] = R(0);
  R ETb = R(0), CTb = R(0), ithb = R(0), hfacb = R(0), Tb = R(0), rhocpb = R(0);
  double rhoHb = 0.0;
  for (int i = 0; i < Q; ++i) abv[i] = out_adj(lh, i, facev[i]);
  for (int i = 0; i < Q; ++i) {
    const R wi = wgt<R, DIM>(i);
    const R cu = cdot<C>(i, u);
    const int face = facev[i];
    const R ab = abv[i];
    R postb = R(0);
    if (face < 0 || (face_flow(P, face) == BC_WALL && face_therm(P, face) == TBC_ADIABATIC)) {
      postb = ab;
    } else {
      // val = hg + (1 - ith)(h_ib - heb)
      const int ib = Lt::opp(i);
      const bool dir = face_therm(P, face) == TBC_DIRICHLET;
      const R Tg = dir ? R(2) * R(face_T(P, face)) - T : T;
      const bool open = face_flow(P, face) == BC_OPEN;
      const R cub = open ? -cu : R(0);
      const R ugug = open ? uu : R(0);
      const R wb = wgt<R, DIM>(ib);
      const R Kg = R(3) * cub + R(4.5) * cub * cub - R(1.5) * ugug;
      const R Kb = -R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
      const R heb = wb * (ET + CT * Kb);
      hb[ib] += ab * (R(1) - ith);
      ithb += -ab * (hpop[ib] - heb);
      const R hebb = -ab * (R(1) - ith);
      const R hgb = ab;
      const R Tgb = hgb * wb * (Eref + rhocp * Kg);
      rhocpb += hgb * wb * Tg * Kg;
      const R Kgb = hgb * wb * rhocp * Tg;
      if (open) {
        const R cubb = Kgb * (R(3) + R(9) * cub);
        for (int d = 0; d < DIM; ++d) ub[d] -= cubb * R(Lt::c(i, d));
        uub += -R(1.5) * Kgb;
      }
      if (dir) {
        if (face == 0)
          gpar[PAR_TFACE] += 2.0 * double(Tgb);
        else
          gpar[PAR_TFACE + 1] += 2.0 * double(Tgb);
        Tb -= Tgb;
      } else {
        Tb += Tgb;
      }
      ETb += hebb * wb;
      CTb += hebb * wb * Kb;
      const R Kbb = hebb * wb * CT;
      const R cub2 = Kbb * (-R(3) + R(9) * cu);
      for (int d = 0; d < DIM; ++d) ub[d] += cub2 * R(Lt::c(i, d));
      uub += -R(1.5) * Kbb;
    }
    if (i == 0) {
      // post = h0 - (h0 - he0) ith + (1 - ith/2) H0 (float64 in the forward)
      const R he0 = R(rhoH - double(Eref) * Td + double(w0) * (double(Eref) * Td - 1.5 * double(rhocp) * Td * double(uu)));
      const R H0 = w0 * rhocp * T * Ddiv;
      hb[0] += postb * (R(1) - ith);
      const R he0b = postb * ith;
      ithb += postb * (he0 - hpop[0]) - R(0.5) * postb * H0;
      const R H0b = postb * (R(1) - R(0.5) * ith);
      rhoHb += double(he0b);
      Tb += he0b * (-Eref + w0 * Eref - R(1.5) * w0 * rhocp * uu);
      rhocpb += he0b * w0 * (-R(1.5) * T * uu) + H0b * w0 * T * Ddiv;
      uub += he0b * w0 * (-R(1.5) * rhocp * T);
      Tb += H0b * w0 * rhocp * Ddiv;
      Ddivb += H0b * w0 * rhocp * T;
    } else {
      const R Ki = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
      const R he = wi * (ET + CT * Ki);
      hb[i] += postb * (R(1) - ith);
      const R heb = postb * ith;
      ithb += postb * (he - hpop[i]);
      hfacb += postb * wi * HD;
      HDb += postb * hfac * wi;
      ETb += heb * wi;
      CTb += heb * wi * Ki;
      const R Kib = heb * wi * CT;
      const R cubb = Kib * (R(3) + R(9) * cu);
      for (int d = 0; d < DIM; ++d) ub[d] += cubb * R(Lt::c(i, d));
      uub += -R(1.5) * Kib;
    }
  }
  ithb += -R(0.5) * hfacb;
  CTb += HDb * Ddiv;
  Ddivb += HDb * CT;
  Tb += ETb * Eref;
  rhocpb += CTb * T;
  Tb += CTb * rhocp;
  const R tauhb = -ithb * ith * ith;
  const R lamb_mix = tauhb * R(3) / Eref;
  rhob += rhocpb * cp;
  const R cpb = rhocpb * rho;
  mixture_adj<R, NP>(lamb_mix, phi, fs, P.lam_s, P.lam_l, phib, fsb);
  mixture_adj<R, NP>(cpb, phi, fs, P.cp_s, P.cp_l, phib, fsb);
  {
    // own T and rho H from the h populations (eq. (H))
    double dT_dH, dT_dphi[NP], dT_dL[NP], dfl_dH, dfl_dphi[NP], dfl_dL[NP];
    invert_grad<NP>(P, phi, rhoH, dT_dH, dT_dphi, dT_dL, dfl_dH, dfl_dphi, dfl_dL);
    const double Tbd = double(Tb);
    rhoHb += Tbd * dT_dH;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      phib[p] += R(Tbd * dT_dphi[p]);
      gpar[PAR_LATENT + p] += Tbd * dT_dL[p];
    }
    for (int i = 0; i < Q; ++i) hb[i] += R(rhoHb);
    qpb += R(0.5 * rhoHb);
  }
  for (int i = 0; i < Q; ++i) blo.st(lh * Q + i, cell, ST(hb[i]));

  // -- phase-field LBs --
  R Ddivb_g = R(0);
  for (int p = 0; p < NP; ++p) {
    const int l = 1 + p;
    R gb[Q], dpub[DIM];
    for (int i = 0; i < Q; ++i) gb[i] = R(0);
    for (int d = 0; d < DIM; ++d) dpub[d] = R(0);
    R phDb = R(0);
    for (int i = 0; i < Q; ++i) abv[i] = out_adj(l, i, facev[i]);
    for (int i = 0; i < Q; ++i) {
      const R wi = wgt<R, DIM>(i);
      const R cu = cdot<C>(i, u);
      const int face = facev[i];
      const R ab = abv[i];
      R postb = R(0);
      if (face < 0 || face_flow(P, face) == BC_WALL) {
        postb = ab;
      } else {
        // val = geb + (1 - itg)(g_ib - geb), geb = w_ib phi (1 - 3 c.u)
        const int ib = Lt::opp(i);
        const R wb = wgt<R, DIM>(ib);
        gb[ib] += ab * (R(1) - itg);
        const R gebb = ab * itg;
        phib[p] += gebb * wb * (R(1) - R(3) * cu);
        const R cub = gebb * wb * phi[p] * (-R(3));
        for (int d = 0; d < DIM; ++d) ub[d] += cub * R(Lt::c(i, d));
      }
      gb[i] += postb * (R(1) - itg);
      const R geb = postb * itg;
      const R Gib = postb * gfac;
      phib[p] += geb * wi * (R(1) + R(3) * cu);
      const R cub = geb * wi * phi[p] * R(3);
      for (int d = 0; d < DIM; ++d) {
        ub[d] += cub * R(Lt::c(i, d));
        dpub[d] += Gib * wi * R(Lt::c(i, d));
      }
      phDb += Gib * wi;
    }
    phib[p] += phDb * Ddiv;
    Ddivb_g += phDb * phi[p];
    for (int d = 0; d < DIM; ++d) {
      phib[p] += R(3) * dpub[d] * u[d];
      ub[d] += R(3) * dpub[d] * phi[p];
      phipb[p] -= R(3) * dpub[d] * uprev[d];
      upb[d] -= R(3) * dpub[d] * phip[p];
      Rpb[p][d] += dpub[d];
    }
    for (int i = 0; i < Q; ++i) blo.st(l * Q + i, cell, ST(gb[i]));
  }
  Ddivb += Ddivb_g;

  // -- flow LB and its face rules --
  R fb[Q];
  for (int i = 0; i < Q; ++i) fb[i] = R(0);
  R sfacb = R(0);
  for (int i = 0; i < Q; ++i) abv[i] = out_adj(0, i, facev[i]);
  for (int i = 0; i < Q; ++i) {
    const R wi = wgt<R, DIM>(i);
    const R cu = cdot<C>(i, u);
    const int face = facev[i];
    const R ab = abv[i];
    R postb = R(0);
    if (face < 0 || face_flow(P, face) == BC_WALL) {
      postb = ab;
    } else {
      // val = rho sb + (1 - itf)(f_ib - feb), feb = 3 p w_ib + rho sb
      const int ib = Lt::opp(i);
      const R cub = -cu;
      const R wb = wgt<R, DIM>(ib);
      const R sb = wb * (R(3) * cub + R(4.5) * cub * cub - R(1.5) * uu);
      const R feb = R(3) * pr * wb + rho * sb;
      rhob += ab * sb;
      R sbb = ab * rho;
      fb[ib] += ab * (R(1) - itf);
      // the cell's own f populations are read again here rather than kept
      // in registers since the forward recompute
      itfb += -ab * (R(bpi.ld(ib, cell)) - feb);
      const R febb = -ab * (R(1) - itf);
      prb += febb * R(3) * wb;
      rhob += febb * sb;
      sbb += febb * rho;
      const R cubb = sbb * wb * (R(3) + R(9) * cub);
      for (int d = 0; d < DIM; ++d) ub[d] -= cubb * R(Lt::c(i, d));
      uub += -R(1.5) * sbb * wb;
    }
    const R cF = cdot<C>(i, Fa);
    const R cFs = cdot<C>(i, F);
    const R c2 = R(Lt::c(i, 0) * Lt::c(i, 0) + Lt::c(i, 1) * Lt::c(i, 1) + Lt::c(i, 2) * Lt::c(i, 2));
    const R qq = R(2) * cu * cFs - R(2.0 / 3.0) * uF + lam_iso * (c2 - R(DIM) * R(1.0 / 3.0));
    const R Fi = wi * (S + R(3) * cF + R(4.5) * qq);
    const R si = wi * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
    const R fe = (i == 0) ? R(3) * pr * (w0 - R(1)) + rho * si : R(3) * pr * wi + rho * si;
    fb[i] += postb * (R(1) - itf);
    const R feb = postb * itf;
    itfb += postb * (fe - R(bpi.ld(i, cell)));
    sfacb += postb * Fi;
    const R Fib = postb * sfac;
    prb += feb * ((i == 0) ? R(3) * (w0 - R(1)) : R(3) * wi);
    rhob += feb * si;
    const R sib = feb * rho;
    R cub = sib * wi * (R(3) + R(9) * cu);
    uub += -R(1.5) * sib * wi;
    Sb += Fib * wi;
    const R cFb = R(3) * Fib * wi;
    const R qqb = R(4.5) * Fib * wi;
    cub += R(2) * qqb * cFs;
    const R cFsb = R(2) * qqb * cu;
    uFb += -R(2.0 / 3.0) * qqb;
    lamb += qqb * (c2 - R(DIM) * R(1.0 / 3.0));
    for (int d = 0; d < DIM; ++d) {
      ub[d] += cub * R(Lt::c(i, d));
      Fab[d] += cFb * R(Lt::c(i, d));
      Fb[d] += cFsb * R(Lt::c(i, d));
    }
  }

  // -- pressure, forcing moments, relaxation time --
  itfb += -R(0.5) * sfacb;
  const R sfb = prb * KP;
  Sb += R(0.5) * prb * KP;
  R taufb = prb * KP * F0;
  const R F0b = prb * KP * (tau_f - R(0.5));
  rhob += prb * KP * s0u;
  const R s0ub = prb * KP * rho;
  uub += -R(1.5) * w0 * s0ub;
  Sb += F0b * w0;
  uFb += -R(3) * w0 * F0b;
  lamb += -R(1.5) * R(DIM) * w0 * F0b;
  for (int i = 1; i < Q; ++i) fb[i] += sfb;
  taufb += -itf * itf * itfb;
  const R mub = R(3) * irho * taufb;
  R irhob = R(3) * mu * taufb;
  mixture_adj<R, NP>(mub, phi, fs, P.mu_s, P.mu_l, phib, fsb);
  rhob += R(2.0 / DIM) * R(1.0 / 3.0) * S * lamb;
  Sb += R(2.0 / DIM) * R(1.0 / 3.0) * rho * lamb;
  for (int d = 0; d < DIM; ++d) {
    ub[d] += uFb * F[d];
    Fb[d] += uFb * u[d];
    ub[d] += R(2) * uub * u[d];
  }
  // S = rho mdot + u . grad rho
  rhob += Sb * mdot;
  const R mdotb = Sb * rho;
  R grhob[DIM];
  for (int d = 0; d < DIM; ++d) {
    ub[d] += Sb * grho[d];
    grhob[d] = Sb * u[d];
  }
  // mdot = -msum / rho
  const R msumb = -mdotb * irho;
  irhob += -mdotb * msum;
  R gfpb[NP][DIM];
  for (int p = 0; p < NP; ++p)
    for (int d = 0; d < DIM; ++d) gfpb[p][d] = R(0);
  for (int p = 0; p < NP; ++p) {
    if (!P.freezes[p]) continue;
    const R dr = R(P.rho_s[p] - P.rho_l[p]);
    fsb += msumb * dr * phi[p];
    phib[p] += msumb * dr * fs;
    fspb -= msumb * dr * phip[p];
    phipb[p] -= msumb * dr * fsp;
    for (int d = 0; d < DIM; ++d) {
      ub[d] += msumb * dr * gfp[p][d];
      gfpb[p][d] += msumb * dr * u[d];
    }
  }
  // u = us (1 - ws/2), Fa = F - rho ws us
  R wsb = R(0), usb[DIM];
  for (int d = 0; d < DIM; ++d) {
    usb[d] = ub[d] * (R(1) - R(0.5) * ws) - Fab[d] * rho * ws;
    wsb += -R(0.5) * ub[d] * us[d] - Fab[d] * rho * us[d];
    Fb[d] += Fab[d];
    rhob += -Fab[d] * ws * us[d];
  }
  // us = (mom + F/2) / rho
  R momb[DIM];
  for (int d = 0; d < DIM; ++d) {
    momb[d] = usb[d] * irho;
    Fb[d] += R(0.5) * usb[d] * irho;
    irhob += usb[d] * (mom[d] + R(0.5) * F[d]);
  }
  fsb += wsb * psi;
  const R psib = wsb * fs;
  for (int p = 0; p < NP; ++p)
    if (P.freezes[p]) phib[p] += psib;
  rhob += -irho * irho * irhob;
  for (int i = 1; i < Q; ++i)
    for (int d = 0; d < DIM; ++d) fb[i] += momb[d] * R(Lt::c(i, d));
  for (int i = 0; i < Q; ++i) blo.st(i, cell, ST(fb[i]));

  // F = sum_p mu_p grad phi_p + rho g
  R mupb[NP], gphib[NP][DIM], lphib[NP];
  for (int p = 0; p < NP; ++p) {
    mupb[p] = R(0);
    lphib[p] = R(0);
    for (int d = 0; d < DIM; ++d) {
      mupb[p] += Fb[d] * gphi[p][d];
      gphib[p][d] = Fb[d] * mup[p];
    }
  }
  for (int d = 0; d < DIM; ++d) rhob += Fb[d] * R(P.grav[d]);

  // -- interface: chemical potentials and pairwise normals --
  for (int p = 0; p < NP; ++p) {
    const R gsp = gsecond(phi[p]);
    for (int q = 0; q < NP; ++q) {
      if (q == p) continue;
      const R gs = gsecond(phi[p] + phi[q]);
      const R b2 = R(2) * R(P.beta[p][q]) * mupb[p];
      phib[p] += b2 * (gsp - gs);
      phib[q] += -b2 * gs;
      lphib[q] += -mupb[p] * R(P.kpq[p][q]);
    }
  }
  for (int p = 0; p < NP; ++p)
    for (int q = p + 1; q < NP; ++q) {
      R v[DIM], vv = R(0);
      for (int d = 0; d < DIM; ++d) {
        v[d] = phi[q] * gphi[p][d] - phi[p] * gphi[q][d];
        vv += v[d] * v[d];
      }
      const R nrm = sqrt(vv + R(1e-24));
      const R A = R(4) * phi[p] * phi[q] * ieps;
      const R sc = A / nrm;
      R vb[DIM], scb = R(0);
      for (int d = 0; d < DIM; ++d) {
        vb[d] = sc * (Rpb[p][d] - Rpb[q][d]);
        scb += (Rpb[p][d] - Rpb[q][d]) * v[d];
      }
      const R Ab = scb / nrm;
      const R nrmb = -scb * A / (nrm * nrm);
      const R vvb = nrmb / (R(2) * nrm);
      for (int d = 0; d < DIM; ++d) vb[d] += R(2) * v[d] * vvb;
      phib[p] += Ab * R(4) * phi[q] * ieps;
      phib[q] += Ab * R(4) * phi[p] * ieps;
      for (int d = 0; d < DIM; ++d) {
        phib[q] += vb[d] * gphi[p][d];
        gphib[p][d] += vb[d] * phi[q];
        phib[p] -= vb[d] * gphi[q][d];
        gphib[q][d] -= vb[d] * phi[p];
      }
    }

  // -- finite differences: own-cell term of the Laplacian; the neighbour
  //    terms are gathered in pass 3 --
  for (int p = 0; p < NP; ++p) phib[p] += -R(6) * (R(1) - w0) * lphib[p];
  // own rho (mixture of own phi, f_s)
  mixture_adj<R, NP>(rhob, phi, fs, P.rho_s, P.rho_l, phib, fsb);

  for (int p = 0; p < NP; ++p) {
    for (int d = 0; d < DIM; ++d) {
      bw.st(L::F_GPHI + p * DIM + d, cell, gphib[p][d]);
      bw.st(L::F_GFP + p * DIM + d, cell, gfpb[p][d]);
    }
    bw.st(L::F_LPHI + p, cell, lphib[p]);
    bw.st(L::O_PHI + p, cell, phib[p]);
    bw.st(L::L_PHI + p, cell, phipb[p]);
  }
  for (int d = 0; d < DIM; ++d) {
    bw.st(L::F_GRHO + d, cell, grhob[d]);
    bw.st(L::L_U + d, cell, upb[d]);
  }
  bw.st(L::F_DIV, cell, Ddivb);
  bw.st(L::O_FS, cell, fsb);
  bw.st(L::L_FS, cell, fspb);
  bw.st(L::L_Q, cell, qpb);
  bw.st(L::M_RHOH, cell, R(rhoH));  // for pass 3 of this cell
}

template <class C>
__host__ __device__ inline void adj_collide_cell(const AdjArgs<C>& a, const KParams& P, int cell, double* gpar) {
  const int area = (int)P.area;
  const int w = cell / area, lat = cell - w * area;
  NbGlobal<C> nb;
  nb.a = &a;
  nb.gx = lat % P.nx;
  nb.gy = lat / P.nx;
  nb.w = w;
  adj_collide_cell<C>(a, P, cell, gpar, nb);
}

// ---------------------------------------------------------------------------
// Pass 3: gather of the finite-difference adjoints from the cells that read
// this cell (and its ghost images), then the reverse of the mixture density,
// the inversion and the moments.  seed = true: the objective's adjoints of
// phi, f_s stand in the own planes and every other input adjoint is zero
// (the populations' adjoints are then written, not added to).
// fda(k, xcell, dl0, dl1, dw) returns work plane k (an FD-adjoint plane) of
// reader cell xcell, which sits at lateral offsets (dl0, dl1) and layer
// offset dw from this cell: from global memory, or from an LDS tile.
// ---------------------------------------------------------------------------
template <class C>
struct FdaGlobal {
  const AdjArgs<C>* a;
  long long nc;
  __host__ __device__ typename C::R operator()(int k, int xcell, int, int, int) const {
    return wplane(*a, k, nc)[xcell];
  }
};

template <class C, class FDA>
__host__ __device__ inline void adj_gather_cell(const AdjArgs<C>& a, const KParams& P, int cell, bool seed,
                                                double* gpar, const FDA& fda) {
  using R = typename C::R;
  using ST = typename C::S;
  using Lt = typename C::L;
  using L = AdjLayout<C>;
  constexpr int Q = C::Q, NP = C::NP, DIM = C::DIM;
  const long long nc = P.ncell;
  const int area = (int)P.area;
  const int w = cell / area, lat = cell - w * area;
  const int gx = lat % P.nx, gy = lat / P.nx;

  R phi[NP];
  for (int p = 0; p < NP; ++p) phi[p] = m_phi<C>(a, p, cell, nc);
  const R fs = m_fs<C>(a, cell, nc);
  const double rhoH = double(wplane(a, L::M_RHOH, nc)[cell]);

  // values read at the end, loaded before any store of this cell
  const R div = R(plane(a.ain, C::A_DIV, nc)[cell]);
  const R lq = seed ? R(0) : wplane(a, L::L_Q, nc)[cell];
  R lphv[NP];
  for (int p = 0; p < NP; ++p) lphv[p] = seed ? R(0) : wplane(a, L::L_PHI + p, nc)[cell];
  const R lfs = seed ? R(0) : wplane(a, L::L_FS, nc)[cell];
  R phib[NP], fsb = wplane(a, L::O_FS, nc)[cell], rhob = R(0), upb[DIM];
  for (int p = 0; p < NP; ++p) phib[p] = wplane(a, L::O_PHI + p, nc)[cell];
  for (int d = 0; d < DIM; ++d) upb[d] = seed ? R(0) : wplane(a, L::L_U + d, nc)[cell];
  if (!seed) {
    for (int p = 0; p < NP; ++p) phib[p] += R(plane(a.lain, p, nc)[cell]);
    fsb += R(plane(a.lain, C::A_FS, nc)[cell]);

    // Contribution of reader x (direction i reads this cell or its ghost
    // image) to the adjoints of the values read: phi, f_s, rho, u^{n-1}.
    auto reader = [&](int xcell, int i, int dw, R* Ab, R& fsrb, R& rhorb, R* uprb, const R* phiread, R fsread) {
      const R wi = wgt<R, DIM>(i);
      const int d0 = -Lt::cl0(i), d1 = -Lt::cl1(i);
      for (int p = 0; p < NP; ++p) {
        R g = R(0), gf = R(0);
        for (int d = 0; d < DIM; ++d) {
          g += R(Lt::c(i, d)) * fda(L::F_GPHI + p * DIM + d, xcell, d0, d1, dw);
          gf += R(Lt::c(i, d)) * fda(L::F_GFP + p * DIM + d, xcell, d0, d1, dw);
        }
        Ab[p] += R(3) * wi * g + R(6) * wi * fda(L::F_LPHI + p, xcell, d0, d1, dw) + R(3) * wi * gf * fsread;
        fsrb += R(3) * wi * gf * phiread[p];
      }
      R gr = R(0);
      for (int d = 0; d < DIM; ++d) gr += R(Lt::c(i, d)) * fda(L::F_GRHO + d, xcell, d0, d1, dw);
      rhorb += R(3) * wi * gr;
      const R db = fda(L::F_DIV, xcell, d0, d1, dw);
      for (int d = 0; d < DIM; ++d) uprb[d] += R(3) * wi * R(Lt::c(i, d)) * db;
    };

    // inner reads: x = y - c_i reads y in direction i
    for (int i = 1; i < Q; ++i) {
      const int xw = w - Lt::cw(i);
      if (xw < 0 || xw >= P.nwn) continue;
      int xl = wrap1(gx - Lt::cl0(i), P.nx);
      if (DIM == 3) xl += wrap1(gy - Lt::cl1(i), P.ny) * P.nx;
      reader(xw * area + xl, i, -Lt::cw(i), phib, fsb, rhob, upb, phi, fs);
    }
    // ghost images: a reader in the boundary layer whose direction leaves
    // through the face reads the ghost derived from this cell
    for (int face = 0; face < 2; ++face) {
      const int bw = face == 0 ? 0 : P.nwn - 1;
      if (w != bw) continue;
      const bool wet = face == 0 && P.flow_bc[0] == BC_WALL;
      R gval[NP];
      for (int p = 0; p < NP; ++p) {
        if (wet) {
          R acc = R(0);
          for (int q = 0; q < NP; ++q)
            if (q != p) acc += phi[p] * phi[q] * R(P.cth[p][q]);
          gval[p] = phi[p] + R(P.four_eps) * acc;
        } else {
          gval[p] = phi[p];
        }
      }
      R Ab[NP], fsgb = R(0), rhogb = R(0), upgb[DIM];
      for (int p = 0; p < NP; ++p) Ab[p] = R(0);
      for (int d = 0; d < DIM; ++d) upgb[d] = R(0);
      for (int i = 1; i < Q; ++i) {
        if (Lt::cw(i) != (face == 0 ? -1 : 1)) continue;
        int xl = wrap1(gx - Lt::cl0(i), P.nx);
        if (DIM == 3) xl += wrap1(gy - Lt::cl1(i), P.ny) * P.nx;
        reader(bw * area + xl, i, 0, Ab, fsgb, rhogb, upgb, gval, fs);
      }
      fsb += fsgb;
      rhob += rhogb;
      const R sgn = face_flow(P, face) == BC_WALL ? R(-1) : R(1);
      for (int d = 0; d < DIM; ++d) upb[d] += sgn * upgb[d];
      if (wet) {
        const R fe = R(P.four_eps);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          phib[p] += Ab[p];
#pragma unroll
          for (int q = 0; q < NP; ++q) {
            if (q == p) continue;
            // d gval_p / d phi_p = 1 + fe sum_q phi_q cth_pq; d gval_p / d phi_q = fe phi_p cth_pq
            phib[p] += Ab[p] * fe * phi[q] * R(P.cth[p][q]);
            phib[q] += Ab[p] * fe * phi[p] * R(P.cth[p][q]);
            gpar[PAR_CTH + p * MAXP + q] += double(Ab[p] * fe * phi[p] * phi[q]);
          }
        }
      } else {
        for (int p = 0; p < NP; ++p) phib[p] += Ab[p];
      }
    }
    mixture_adj<R, NP>(rhob, phi, fs, P.rho_s, P.rho_l, phib, fsb);
  }

  // f_s = 1 - f_l(phi, rho H); phi = sum g / (1 - D/2); rho H = sum h + q/2
  double dT_dH, dT_dphi[NP], dT_dL[NP], dfl_dH, dfl_dphi[NP], dfl_dL[NP];
  invert_grad<NP>(P, phi, rhoH, dT_dH, dT_dphi, dT_dL, dfl_dH, dfl_dphi, dfl_dL);
  const double flb = -double(fsb);
  const double rhoHb = flb * dfl_dH;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    phib[p] += R(flb * dfl_dphi[p]);
    gpar[PAR_LATENT + p] += flb * dfl_dL[p];
  }
  const R idiv = R(1) / (R(1) - R(0.5) * div);
  R Db = R(0);
  for (int p = 0; p < NP; ++p) {
    Db += phib[p] * phi[p] * R(0.5) * idiv;
    plane(a.laout, AdjScal<C>::GS + p, nc)[cell] = ST(phib[p] * idiv);
  }
  plane(a.laout, AdjScal<C>::HS, nc)[cell] = ST(R(rhoHb));
  if (seed)
    for (int k = 0; k < (NP + 2) * Q; ++k) plane(a.lpout, k, nc)[cell] = ST(0);
  const R qb = lq + R(0.5 * rhoHb);
  for (int p = 0; p < NP; ++p) plane(a.laout, p, nc)[cell] = ST(lphv[p]);
  plane(a.laout, C::A_FS, nc)[cell] = ST(lfs);
  for (int d = 0; d < DIM; ++d) plane(a.laout, C::A_U + d, nc)[cell] = ST(upb[d]);
  plane(a.laout, C::A_DIV, nc)[cell] = ST(Db);
  plane(a.laout, C::A_Q, nc)[cell] = ST(qb);
}

template <class C>
__host__ __device__ inline void adj_gather_cell(const AdjArgs<C>& a, const KParams& P, int cell, bool seed,
                                                double* gpar) {
  FdaGlobal<C> g;
  g.a = &a;
  g.nc = P.ncell;
  adj_gather_cell<C>(a, P, cell, seed, gpar, g);
}

// Objectives of the final state, both of the form J = A / D with
// A = sum f_s psi over cells (psi the freezing phases' fraction):
//   frozen fraction  D = sum psi:                shift = A / D, scale = 1 / D
//   front position   D = cells per wall layer:   shift = 0,     scale = 1 / D
// (the volume-equivalent solid thickness).  Adjoints of phi_p (freezing
// phases) and f_s into the own planes: dJ/dphi_p = (f_s - shift) scale,
// dJ/df_s = psi scale.
template <class C>
__host__ __device__ inline void adj_seed_cell(const AdjArgs<C>& a, const KParams& P, int cell, double shift,
                                              double scale) {
  using R = typename C::R;
  using L = AdjLayout<C>;
  constexpr int NP = C::NP;
  const long long nc = P.ncell;
  R psi = R(0);
  for (int p = 0; p < NP; ++p)
    if (P.freezes[p]) psi += wplane(a, L::M_PHI + p, nc)[cell];
  const R fs = wplane(a, L::M_FS, nc)[cell];
  for (int p = 0; p < NP; ++p)
    wplane(a, L::O_PHI + p, nc)[cell] = P.freezes[p] ? R((double(fs) - shift) * scale) : R(0);
  wplane(a, L::O_FS, nc)[cell] = R(double(psi) * scale);
}

// Dependence of the initial state on the latent heats: the rest enthalpy
// population of a liquid cell holds rho H = rho_l C_l T + sum_p phi_p
// rho_p^l L_p.  Adds sum over cells lambda_{h,0} phi_p rho_p^l (1 - f_s).
template <class C>
__host__ __device__ inline void adj_init_latent_cell(const AdjArgs<C>& a, const KParams& P, int cell,
                                                     double* gpar) {
  constexpr int Q = C::Q, NP = C::NP;
  const long long nc = P.ncell;
  const double lh0 = double(adj_pop<C>(a.lpin, a.lain, NP + 1, 0, cell, nc));
  const double fl = 1.0 - double(plane(a.ain, C::A_FS, nc)[cell]);
#pragma unroll
  for (int p = 0; p < NP; ++p)
    gpar[PAR_LATENT + p] += lh0 * fl * double(plane(a.ain, p, nc)[cell]) * P.rho_l[p];
}

}  // namespace lbf
