// Host-side parameter validation, derived kernel parameters and the layout
// of the caller-provided state buffer.
#pragma once

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "../../include/lbfreeze.h"
#include "lbf_lattice.h"

namespace lbf {

inline bool all_finite(const double* a, long long n) {
  for (long long k = 0; k < n; ++k)
    if (!isfinite(a[k])) return false;
  return true;
}

inline int lattice_q(int dim) { return dim == 2 ? 9 : 19; }

// Validation of lbf_check_params; returns an empty string when valid.
inline std::string check_params(const lbf_params* P) {
  char buf[256];
  if (!P) return "params is NULL";
  if (P->dim != 2 && P->dim != 3) return "dim must be 2 or 3";
  const int nz = P->dim == 3 ? P->nz : 1;
  if (P->nx < 1 || P->ny < 1 || nz < 1) return "grid sizes must be positive";
  const int nwn = P->dim == 3 ? nz : P->ny;
  if (nwn < 2) return "the wall-normal axis needs at least 2 cells";
  const long long ncell = (long long)P->nx * P->ny * nz;
  if (ncell > (1LL << 31) / 2) return "grid too large (cell index exceeds 2^30)";
  if ((long long)P->nx * (P->dim == 3 ? P->ny : 1) > (1LL << 30)) return "layer too large";
  if (P->nphase < 1 || P->nphase > LBF_MAXP) return "nphase must be 1..4";
  if (P->precision != LBF_FP32 && P->precision != LBF_FP64 && P->precision != LBF_MIXED)
    return "precision must be LBF_FP32, LBF_FP64 or LBF_MIXED";
  for (int f = 0; f < 2; ++f) {
    if (P->flow_bc[f] != LBF_BC_WALL && P->flow_bc[f] != LBF_BC_OPEN) return "flow_bc must be WALL or OPEN";
    if (P->therm_bc[f] != LBF_TBC_DIRICHLET && P->therm_bc[f] != LBF_TBC_ADIABATIC)
      return "therm_bc must be DIRICHLET or ADIABATIC";
    if (!isfinite(P->T_face[f])) return "T_face must be finite";
  }
  if (!(P->eps > 0) || !isfinite(P->eps)) return "eps must be positive";
  if (!(P->tau_g > 0.5) || !isfinite(P->tau_g)) return "tau_g must exceed 1/2";
  if (!(P->E_ref > 0) || !isfinite(P->E_ref)) return "E_ref must be positive";
  if (!isfinite(P->T_melt)) return "T_melt must be finite";
  for (int a = 0; a < 3; ++a)
    if (!isfinite(P->gravity[a])) return "gravity must be finite";
  const double w0 = P->dim == 2 ? 4.0 / 9.0 : 1.0 / 3.0;
  for (int p = 0; p < P->nphase; ++p) {
    const double vals[9] = {P->rho_l[p], P->rho_s[p], P->mu_l[p], P->mu_s[p], P->lam_l[p],
                            P->lam_s[p], P->cp_l[p], P->cp_s[p], P->latent[p]};
    for (double v : vals)
      if (!isfinite(v)) return "material properties must be finite";
    if (!(P->rho_l[p] > 0 && P->rho_s[p] > 0)) return "densities must be positive";
    if (!(P->cp_l[p] > 0 && P->cp_s[p] > 0)) return "heat capacities must be positive";
    if (!(P->mu_l[p] > 0 && P->mu_s[p] > 0)) return "viscosities must be positive";
    if (!(P->lam_l[p] > 0 && P->lam_s[p] > 0)) return "conductivities must be positive";
    if (P->latent[p] < 0) return "latent heat must be non-negative";
    if (P->freezes[p] != 0 && P->freezes[p] != 1) return "freezes must be 0 or 1";
    if (!P->freezes[p]) {
      if (P->rho_l[p] != P->rho_s[p] || P->mu_l[p] != P->mu_s[p] || P->lam_l[p] != P->lam_s[p] ||
          P->cp_l[p] != P->cp_s[p] || P->latent[p] != 0.0) {
        snprintf(buf, sizeof buf, "phase %d does not freeze but has distinct solid values or L > 0", p);
        return buf;
      }
    }
    // relaxation times of the pure phase in both states
    const double tf_l = 3.0 * P->mu_l[p] / P->rho_l[p] + 0.5, tf_s = 3.0 * P->mu_s[p] / P->rho_s[p] + 0.5;
    const double th_l = 3.0 * P->lam_l[p] / P->E_ref + 0.5, th_s = 3.0 * P->lam_s[p] / P->E_ref + 0.5;
    if (!(tf_l > 0.5 && tf_s > 0.5 && th_l > 0.5 && th_s > 0.5)) {
      snprintf(buf, sizeof buf, "phase %d: relaxation time not above 1/2", p);
      return buf;
    }
    // non-negative rest weight of the enthalpy equilibrium
    const double lim = (1.0 - w0) * P->E_ref * (1.0 - 1e-12);
    if (P->rho_l[p] * P->cp_l[p] < lim || P->rho_s[p] * P->cp_s[p] < lim) {
      snprintf(buf, sizeof buf, "phase %d: rho C_p below (1 - w_0) E_ref", p);
      return buf;
    }
  }
  for (int p = 0; p < P->nphase; ++p)
    for (int q = 0; q < P->nphase; ++q) {
      if (!isfinite(P->sigma[p][q]) || !isfinite(P->cos_theta[p][q])) return "sigma/cos_theta must be finite";
      if (p != q && P->sigma[p][q] != P->sigma[q][p]) return "sigma must be symmetric";
      if (p != q && P->sigma[p][q] < 0) return "sigma must be non-negative";
      if (P->cos_theta[p][q] != -P->cos_theta[q][p]) return "cos_theta must be antisymmetric";
      if (fabs(P->cos_theta[p][q]) > 1.0) return "|cos_theta| must be <= 1";
    }
  return "";
}

inline KParams make_kparams(const lbf_params* P) {
  KParams k;
  memset(&k, 0, sizeof k);
  k.nx = P->nx;
  k.ny = P->ny;
  k.nz = P->dim == 3 ? P->nz : 1;
  k.nwn = P->dim == 3 ? k.nz : k.ny;
  k.area = P->dim == 3 ? (long long)k.nx * k.ny : (long long)k.nx;
  k.ncell = (long long)k.nx * k.ny * k.nz;
  for (int f = 0; f < 2; ++f) {
    k.flow_bc[f] = P->flow_bc[f];
    k.therm_bc[f] = P->therm_bc[f];
    k.T_face[f] = P->T_face[f];
  }
  for (int p = 0; p < P->nphase; ++p) {
    k.freezes[p] = P->freezes[p];
    k.rho_l[p] = P->rho_l[p];
    k.rho_s[p] = P->rho_s[p];
    k.mu_l[p] = P->mu_l[p];
    k.mu_s[p] = P->mu_s[p];
    k.lam_l[p] = P->lam_l[p];
    k.lam_s[p] = P->lam_s[p];
    k.cp_l[p] = P->cp_l[p];
    k.cp_s[p] = P->cp_s[p];
    k.latent[p] = P->latent[p];
    for (int q = 0; q < P->nphase; ++q) {
      k.beta[p][q] = 3.0 * P->sigma[p][q] / P->eps;
      k.kpq[p][q] = -0.75 * P->eps * P->sigma[p][q];
      k.cth[p][q] = P->cos_theta[p][q];
    }
  }
  k.eps = P->eps;
  k.four_eps = 4.0 / P->eps;
  k.tau_g = P->tau_g;
  k.T_melt = P->T_melt;
  k.E_ref = P->E_ref;
  for (int a = 0; a < 3; ++a) k.grav[a] = a < P->dim ? P->gravity[a] : 0.0;
  return k;
}

// Layout of the caller-provided device buffer (256-byte aligned pieces).
struct Layout {
  size_t elt;          // bytes per stored value
  size_t pop_bytes;    // one population buffer
  size_t aux_bytes;    // one lagged-field buffer
  size_t off_pop[2], off_aux[2], off_stage, off_part, off_out, off_kp, total;
  int nv;              // diagnostic values
};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

inline Layout make_layout(const lbf_params* P) {
  Layout L;
  const long long ncell = (long long)P->nx * P->ny * (P->dim == 3 ? P->nz : 1);
  const int Q = lattice_q(P->dim), N = P->nphase;
  L.elt = P->precision == LBF_FP64 ? 8 : 4;
  L.pop_bytes = (size_t)(N + 2) * Q * ncell * L.elt;
  L.aux_bytes = (size_t)(N + P->dim + 3) * ncell * L.elt;
  L.nv = 3 * N + 4;
  size_t o = 0;
  for (int k = 0; k < 2; ++k) {
    L.off_pop[k] = o;
    o = align256(o + L.pop_bytes);
  }
  for (int k = 0; k < 2; ++k) {
    L.off_aux[k] = o;
    o = align256(o + L.aux_bytes);
  }
  L.off_stage = o;
  o = align256(o + (size_t)ncell * 8);
  L.off_part = o;
  o = align256(o + (size_t)DIAG_MAX_BLOCKS * L.nv * 8);
  L.off_out = o;
  o = align256(o + (size_t)L.nv * 8);
  L.off_kp = o;
  o = align256(o + sizeof(KParams));
  L.total = o;
  return L;
}

// Layout of the caller-provided buffer of the reverse step: two adjoint
// states (populations, lagged fields), the work planes of the three passes
// (arithmetic type), per-block partial sums, the gradient accumulator and
// the objective sums.
struct AdjBufLayout {
  size_t off_lp[2], off_la[2], off_work, off_part, off_acc, off_obj, total;
  int nblocks;  // rows of the gradient accumulator: covers every adjoint grid
  int cblocks;  // blocks of the one-thread-per-cell passes (256 cells each)
  int nwork;
};

inline int adj_nwork(int N, int D) { return 2 * N * D + 4 * N + 2 * D + 6; }

inline AdjBufLayout make_adj_layout(const lbf_params* P, const Layout& F) {
  AdjBufLayout A;
  const long long ncell = (long long)P->nx * P->ny * (P->dim == 3 ? P->nz : 1);
  const size_t relt = P->precision == LBF_FP32 ? 4 : 8;
  A.cblocks = (int)((ncell + 255) / 256);
  // The tiled gather's grid: 128-cell rows and chunks of at least two
  // layers (2D), at most ceil(nx / 128) * ceil(nwn / 2) blocks.
  const long long nwn = P->dim == 3 ? P->nz : P->ny;
  // the tiled passes: 128-cell rows, chunks of at least two layers
  const long long tiles = ((long long)(P->nx + 127) / 128) * ((nwn + 1) / 2);
  A.nblocks = (int)(tiles > A.cblocks ? tiles : A.cblocks);
  A.nwork = adj_nwork(P->nphase, P->dim);
  size_t o = 0;
  for (int k = 0; k < 2; ++k) {
    A.off_lp[k] = o;
    o = align256(o + F.pop_bytes);
  }
  // adjoint of the lagged fields plus N + 1 per-cell population scalars
  const size_t la_bytes = F.aux_bytes + (size_t)(P->nphase + 1) * ncell * F.elt;
  for (int k = 0; k < 2; ++k) {
    A.off_la[k] = o;
    o = align256(o + la_bytes);
  }
  A.off_work = o;
  o = align256(o + (size_t)A.nwork * ncell * relt);
  A.off_part = o;
  o = align256(o + (size_t)A.nblocks * 22 * 8 + (size_t)A.cblocks * 2 * 8);
  A.off_acc = o;
  o = align256(o + 22 * 8);
  A.off_obj = o;
  o = align256(o + 2 * 8);
  A.total = o;
  return A;
}

}  // namespace lbf
