// Host emulator of the reverse (adjoint) step (test support for the HIP
// path): runs the adjoint pass functions of lbf_adjoint.h on the CPU over a
// whole forward trajectory held in memory, so that the CPU tests can check
// the hand-written adjoint against finite differences of the forward step
// and of the oracle.  Not part of the library's compute path.
#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/lbfreeze.h"
#include "lbf_adjoint.h"
#include "lbf_adjoint_kernels.h"
#include "lbf_host.h"
#include "lbf_kernels.h"

namespace {

using namespace lbf;

template <class C>
void forward_step(std::vector<typename C::S>& popA, std::vector<typename C::S>& auxA,
                  std::vector<typename C::S>& popB, std::vector<typename C::S>& auxB, const KParams& P) {
  StepArgs<typename C::S> a;
  memset(&a, 0, sizeof a);
  a.pin = popA.data();
  a.pout = popB.data();
  a.ain = auxA.data();
  a.aout = auxB.data();
  const Geometry g = step_geometry<C>(P);
  a.ntx = g.ntx;
  a.nty = g.nty;
  a.chunk = g.chunk;
  a.nblocks = g.nblocks;
  a.mom = a.aout;
  for (int cell = 0; cell < (int)P.ncell; ++cell) moment_cell<C>(a, P, cell);
  std::vector<Smem<C>> smv(1);
  Smem<C>& sm = smv[0];
  for (int b = 0; b < g.nblocks; ++b) {
    const BlockPos bp = block_pos<C>(a, P, b);
    if (bp.w0 == 0) {
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(a, P, sm, bp, f, 0);
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(a, P, sm, bp, f, -1);
    } else {
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(a, P, sm, bp, f, bp.w0 - 1);
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(a, P, sm, bp, f, bp.w0);
    }
    for (int w = bp.w0; w < bp.w1; ++w) {
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(a, P, sm, bp, f, w + 1);
      const bool edge = (w == 0 || w == P.nwn - 1);
      for (int t = 0; t < C::NT; ++t) {
        if (edge)
          process_cell<C, false, true>(a, P, sm, bp, t, w);
        else
          process_cell<C, false, false>(a, P, sm, bp, t, w);
      }
    }
  }
}

// A = sum f_s psi and B = sum psi of a state, from the moments.
template <class C>
void objective_sums(const AdjArgs<C>& a, const KParams& P, double& A, double& B) {
  using L = AdjLayout<C>;
  const long long nc = P.ncell;
  A = B = 0.0;
  for (long long c = 0; c < nc; ++c) {
    double psi = 0.0;
    for (int p = 0; p < C::NP; ++p)
      if (P.freezes[p]) psi += double(wplane(a, L::M_PHI + p, nc)[c]);
    A += double(wplane(a, L::M_FS, nc)[c]) * psi;
    B += psi;
  }
}

// The tiled gather of adj_gather_tile_kernel, block by block, each barrier
// phase for all threads before the next.
template <class C>
void gather_tiled(const AdjArgs<C>& a, const KParams& P, double* gpar) {
  const Geometry g = step_geometry<C>(P);
  StepArgs<typename C::S> sa;
  memset(&sa, 0, sizeof sa);
  sa.ntx = g.ntx;
  sa.nty = g.nty;
  sa.chunk = g.chunk;
  sa.nblocks = g.nblocks;
  std::vector<FdaRing<C>> rv(1);
  FdaRing<C>& ring = rv[0];
  for (int b = 0; b < g.nblocks; ++b) {
    memset(&ring, 0xff, sizeof ring);  // poison: a read of an unfilled slot shows up as NaN
    const BlockPos bp = block_pos<C>(sa, P, b);
    if (bp.w0 > 0)
      for (int f = 0; f < C::F; ++f) fda_fill<C>(a, P, ring, bp, f, bp.w0 - 1);
    for (int f = 0; f < C::F; ++f) fda_fill<C>(a, P, ring, bp, f, bp.w0);
    for (int w = bp.w0; w < bp.w1; ++w) {
      if (w + 1 < P.nwn)
        for (int f = 0; f < C::F; ++f) fda_fill<C>(a, P, ring, bp, f, w + 1);
      for (int t = 0; t < C::NT; ++t) {
        const int tx = t % C::TX, ty = t / C::TX;
        const int gx = bp.tx0 + tx, gy = bp.ty0 + ty;
        if (gx >= P.nx || (C::DIM == 3 && gy >= P.ny)) continue;
        FdaLds<C> acc;
        acc.ring = &ring;
        acc.fc = (C::DIM == 3) ? (ty + 1) * C::LX + tx + 1 : tx + 1;
        acc.w = w;
        const int cell = w * (int)P.area + ((C::DIM == 3) ? gy * P.nx + gx : gx);
        adj_gather_cell<C>(a, P, cell, false, gpar, acc);
      }
    }
  }
}

// The tiled collide reverse of adj_collide_tile_kernel, block by block, each
// barrier phase for all threads before the next.
template <class C>
void collide_tiled(const AdjArgs<C>& a, const KParams& P, double* gpar) {
  const Geometry g = step_geometry<C>(P);
  const StepArgs<typename C::S> sa = fill_args<C>(a, g.ntx, g.nty, g.chunk, g.nblocks);
  std::vector<Smem<C>> smv(1);
  Smem<C>& sm = smv[0];
  for (int b = 0; b < g.nblocks; ++b) {
    memset(&sm, 0xff, sizeof sm);  // poison: a read of an unfilled slot shows up as NaN
    const BlockPos bp = block_pos<C>(sa, P, b);
    if (bp.w0 == 0) {
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(sa, P, sm, bp, f, 0);
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(sa, P, sm, bp, f, -1);
    } else {
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(sa, P, sm, bp, f, bp.w0 - 1);
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(sa, P, sm, bp, f, bp.w0);
    }
    for (int w = bp.w0; w < bp.w1; ++w) {
      for (int f = 0; f < C::F; ++f) fill_layer_cell<C>(sa, P, sm, bp, f, w + 1);
      for (int t = 0; t < C::NT; ++t) {
        const int tx = t % C::TX, ty = t / C::TX;
        const int gx = bp.tx0 + tx, gy = bp.ty0 + ty;
        if (gx >= P.nx || (C::DIM == 3 && gy >= P.ny)) continue;
        NbLds<C> nb;
        nb.sm = &sm;
        nb.fc = (C::DIM == 3) ? (ty + 1) * C::LX + tx + 1 : tx + 1;
        nb.w = w;
        const int cell = w * (int)P.area + ((C::DIM == 3) ? gy * P.nx + gx : gx);
        adj_collide_cell<C>(a, P, cell, gpar, nb);
      }
    }
  }
}

template <int DIM, int NP, typename S, typename R>
int run(const lbf_params* prm, const double* phi, const double* T, int nsteps, int objective, double* J,
        double* grad) {
  using C = CfgOf<DIM, NP, S, R>;
  const KParams P = make_kparams(prm);
  const long long nc = P.ncell;
  const int Q = Lat<DIM>::Q;
  const size_t npop = (size_t)(NP + 2) * Q * nc, naux = (size_t)(NP + DIM + 3) * nc;
  std::vector<double> fields((size_t)(NP + 1) * nc);
  memcpy(fields.data(), phi, (size_t)NP * nc * 8);
  memcpy(fields.data() + (size_t)NP * nc, T, (size_t)nc * 8);
  // the whole trajectory: states x^0 .. x^nsteps
  std::vector<std::vector<S>> pops(nsteps + 1, std::vector<S>(npop)), auxs(nsteps + 1, std::vector<S>(naux));
  for (long long c = 0; c < nc; ++c) init_cell<DIM, NP, S>(P, fields.data(), 0, 0, pops[0].data(), auxs[0].data(), c);
  for (int s = 0; s < nsteps; ++s) forward_step<C>(pops[s], auxs[s], pops[s + 1], auxs[s + 1], P);

  std::vector<R> work((size_t)AdjLayout<C>::NWORK * nc);
  const size_t nla = (size_t)AdjScal<C>::NLA * nc;
  std::vector<S> lpA(npop), laA(nla), lpB(npop), laB(nla);
  std::vector<double> gpar(NPAR, 0.0);
  AdjArgs<C> a;
  a.work = work.data();
  // seed from the final state
  a.pin = pops[nsteps].data();
  a.ain = auxs[nsteps].data();
  a.mom = nullptr;
  a.lpin = nullptr;
  a.lain = nullptr;
  a.lpout = lpA.data();
  a.laout = laA.data();
  for (int c = 0; c < (int)nc; ++c) adj_moment_cell<C>(a, P, c);
  double A, B;
  objective_sums<C>(a, P, A, B);
  const double D = objective == LBF_OBJ_FRONT ? double(P.area) : B;
  const double shift = objective == LBF_OBJ_FRONT ? 0.0 : A / D;
  *J = A / D;
  for (int c = 0; c < (int)nc; ++c) adj_seed_cell<C>(a, P, c, shift, 1.0 / D);
  for (int c = 0; c < (int)nc; ++c) adj_gather_cell<C>(a, P, c, true, gpar.data());
  for (int s = nsteps - 1; s >= 0; --s) {
    a.pin = pops[s].data();
    a.ain = auxs[s].data();
    a.lpin = lpA.data();
    a.lain = laA.data();
    a.lpout = lpB.data();
    a.laout = laB.data();
    std::fill(lpB.begin(), lpB.end(), S(NAN));
    std::fill(laB.begin(), laB.end(), S(NAN));
    // moments of x^n from x^{n+1}'s lagged fields on odd steps, recomputed on
    // even ones: both routes are checked
    a.mom = (s & 1) ? auxs[s + 1].data() : nullptr;
    if (!a.mom)
      for (int c = 0; c < (int)nc; ++c) adj_moment_cell<C>(a, P, c);
    // the tiled collide reverse of the GPU kernel on every third step (from
    // x^{n+1}'s moments or the recomputed ones, by the parity above), the
    // per-cell one otherwise
    if (s % 3 == 1)
      collide_tiled<C>(a, P, gpar.data());
    else
      for (int c = 0; c < (int)nc; ++c) adj_collide_cell<C>(a, P, c, gpar.data());
    // the tiled gather of the GPU kernel on every third step, the plain one
    // otherwise: both are checked
    if (s % 3 == 2)
      gather_tiled<C>(a, P, gpar.data());
    else
      for (int c = 0; c < (int)nc; ++c) adj_gather_cell<C>(a, P, c, false, gpar.data());
    lpA.swap(lpB);
    laA.swap(laB);
  }
  a.pin = pops[0].data();
  a.ain = auxs[0].data();
  a.mom = nullptr;
  a.lpin = lpA.data();
  a.lain = laA.data();
  for (int c = 0; c < (int)nc; ++c) adj_init_latent_cell<C>(a, P, c, gpar.data());
  for (int k = 0; k < NPAR; ++k) grad[k] = gpar[k];
  // as lbf_adjoint_gradient: a non-finite gradient is reported, not returned silently
  return all_finite(grad, NPAR) && isfinite(*J) ? 0 : LBF_ENAN;
}

template <int DIM, typename S, typename R>
int run_n(const lbf_params* prm, const double* phi, const double* T, int nsteps, int objective, double* J,
          double* grad) {
  switch (prm->nphase) {
    case 1: return run<DIM, 1, S, R>(prm, phi, T, nsteps, objective, J, grad);
    case 2: return run<DIM, 2, S, R>(prm, phi, T, nsteps, objective, J, grad);
    case 3: return run<DIM, 3, S, R>(prm, phi, T, nsteps, objective, J, grad);
    case 4: return run<DIM, 4, S, R>(prm, phi, T, nsteps, objective, J, grad);
  }
  return -1;
}

}  // namespace

// Objective J (LBF_OBJ_FROZEN_FRACTION or LBF_OBJ_FRONT) after nsteps from
// an equilibrium start (phi, T; u = 0, p = 0) and its gradient:
// grad[0..1] d J / d T_face, grad[2..5] d J / d L_p, grad[6..21]
// d J / d cth[p][q] (row-major, MAXP x MAXP).
extern "C" int lbf_emu_adjoint(const lbf_params* prm, const double* phi, const double* T, int nsteps,
                               int objective, double* J, double* grad) {
  if (!check_params(prm).empty() || nsteps < 0) return -1;
  if (objective != LBF_OBJ_FROZEN_FRACTION && objective != LBF_OBJ_FRONT) return -3;
  lbf_params q = *prm;
  if (q.dim == 2) q.nz = 1;
  if (q.dim == 2 && q.precision == LBF_FP64) return run_n<2, double, double>(&q, phi, T, nsteps, objective, J, grad);
  if (q.dim == 2 && q.precision == LBF_FP32) return run_n<2, float, float>(&q, phi, T, nsteps, objective, J, grad);
  if (q.dim == 3 && q.precision == LBF_FP64) return run_n<3, double, double>(&q, phi, T, nsteps, objective, J, grad);
  if (q.dim == 3 && q.precision == LBF_FP32) return run_n<3, float, float>(&q, phi, T, nsteps, objective, J, grad);
  return -2;
}

#ifdef LBF_EMU_ADJ_MAIN
#include <stdio.h>

// Sanitizer driver of the reverse step: 2D, every phase count, float64 and
// float32, three face combinations, the frozen-fraction and front objectives
// in turn, on a narrow grid and on one that spans two 128-wide row tiles.
// Four steps reach the per-cell and both tiled forms of the passes.  The
// start has separated phases (a droplet with a core and, for N = 4, a
// bubble): where two phases are mixed in bulk, the pairwise normal is
// rounding noise and its exact derivative overflows float32.  Exit status 0
// when every J and gradient stays finite.
int main() {
  int bad = 0, runs = 0;
  const int shapes[2][2] = {{37, 11}, {150, 21}};
  for (int sh = 0; sh < 2; ++sh)
    for (int N = 1; N <= 4; ++N)
      for (int prec = 0; prec < 2; ++prec)
        for (int bcase = 0; bcase < 3; ++bcase) {
          const int obj = (N + prec + bcase) % 2 ? LBF_OBJ_FRONT : LBF_OBJ_FROZEN_FRACTION;
          lbf_params P;
          memset(&P, 0, sizeof P);
          P.dim = 2;
          P.nx = shapes[sh][0];
          P.ny = shapes[sh][1];
          P.nz = 1;
          P.nphase = N;
          P.precision = prec == 0 ? LBF_FP64 : LBF_FP32;
          P.flow_bc[0] = LBF_BC_WALL;
          P.flow_bc[1] = bcase == 1 ? LBF_BC_OPEN : LBF_BC_WALL;
          P.therm_bc[0] = LBF_TBC_DIRICHLET;
          P.therm_bc[1] = bcase == 2 ? LBF_TBC_DIRICHLET : LBF_TBC_ADIABATIC;
          P.T_face[0] = -0.05;
          P.T_face[1] = 0.05;
          for (int p = 0; p < N; ++p) {
            const bool fr = (p % 2) == 0;
            P.rho_l[p] = fr ? 1.0 : 0.01 * (p + 1);
            P.rho_s[p] = fr ? 0.9 + 0.1 * p : P.rho_l[p];
            P.mu_l[p] = 0.1 * P.rho_l[p];
            P.mu_s[p] = 0.1 * P.rho_s[p];
            P.lam_l[p] = P.lam_s[p] = 0.1;
            P.cp_l[p] = P.cp_s[p] = fr ? 1.0 : 1.0 / P.rho_l[p];
            P.latent[p] = fr ? 1.0 : 0.0;
            P.freezes[p] = fr ? 1 : 0;
            for (int q = 0; q < N; ++q) {
              P.sigma[p][q] = p == q ? 0.0 : 1e-3;
              P.cos_theta[p][q] = p < q ? 0.3 : (p > q ? -0.3 : 0.0);
            }
          }
          P.eps = 4;
          P.tau_g = 0.8;
          P.T_melt = 0;
          P.E_ref = 1;
          const long long nc = (long long)P.nx * P.ny;
          std::vector<double> phi((size_t)N * nc), T(nc);
          for (long long c = 0; c < nc; ++c) {
            const int x = c % P.nx, y = c / P.nx;
            const double r = sqrt((x - 18.0) * (x - 18.0) + (double)y * y);
            const double d = 0.5 + 0.5 * tanh((8.0 - r) / 2.0);
            const double core = 0.5 + 0.5 * tanh((4.0 - r) / 2.0);
            const double rb = sqrt((x - 30.0) * (x - 30.0) + (y - 7.0) * (y - 7.0));
            const double bub = N == 4 ? 0.5 + 0.5 * tanh((2.5 - rb) / 2.0) : 0.0;
            double part[4] = {1.0, 0.0, 0.0, 0.0};
            if (N == 2) {
              part[0] = d;
              part[1] = 1.0 - d;
            } else if (N >= 3) {
              part[0] = d * (1.0 - core);
              part[1] = 1.0 - d;
              part[2] = d * core;
            }
            if (N == 4) {
              for (int p = 0; p < 3; ++p) part[p] *= 1.0 - bub;
              part[3] = bub;
            }
            for (int p = 0; p < N; ++p) phi[(size_t)p * nc + c] = part[p];
            T[c] = 0.005 + 0.002 * y;  // just above melting, cold wall below
          }
          double J = 0.0, g[22];
          const int rc = lbf_emu_adjoint(&P, phi.data(), T.data(), 4, obj, &J, g);
          ++runs;
          bool ok = rc == 0 && isfinite(J);
          for (double v : g) ok = ok && isfinite(v);
          if (!ok) {
            printf("non-finite or refused: %dx%d N=%d prec=%d bc=%d obj=%d rc=%d\n", P.nx, P.ny, N, prec, bcase,
                   obj, rc);
            ++bad;
          }
        }
  printf("%d runs, %d with non-finite output\n", runs, bad);
  return bad ? 1 : 0;
}
#endif
