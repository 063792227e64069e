// Host emulator of the step kernels (test support for the HIP path).
//
// Runs the very phase functions of the moments and collide kernels on the
// CPU: the moments pass cell by cell, then the collide pass block by block,
// with each barrier-separated phase executed for every thread index before
// the next phase starts.  The CPU tests use it to check the kernel's tiling,
// halo, ghost-layer and push-streaming logic against the oracle on small
// grids, and to run the same code under the host address sanitizer, before
// any of it reaches a GPU.  It is not part of the library's compute path.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/lbfreeze.h"
#include "lbf_host.h"
#include "lbf_kernels.h"

namespace {

using namespace lbf;

template <class C, bool M>
void emulate_step(StepArgs<typename C::S> a, const KParams& P) {
  const Geometry g = step_geometry<C>(P);
  a.ntx = g.ntx;
  a.nty = g.nty;
  a.chunk = g.chunk;
  a.nblocks = g.nblocks;
  a.mom = a.aout;
  for (int cell = 0; cell < (int)P.ncell; ++cell) moment_cell<C>(a, P, cell);
  std::unique_ptr<Smem<C>> smp(new Smem<C>());
  Smem<C>& sm = *smp;
  for (int b = 0; b < g.nblocks; ++b) {
    memset(&sm, 0xff, sizeof sm);  // poison: a read of an unfilled slot shows up as NaN
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
          process_cell<C, M, true>(a, P, sm, bp, t, w);
        else
          process_cell<C, M, false>(a, P, sm, bp, t, w);
      }
    }
  }
}

template <int DIM, int NP, typename R, typename RC>
int run(const lbf_params* prm, const double* phi, const double* T, const double* u, const double* p,
        int nsteps, double* pop_out, double* aux_out, double* mom_out) {
  using C = CfgOf<DIM, NP, R, RC>;
  const KParams P = make_kparams(prm);
  const long long nc = P.ncell;
  const int Q = Lat<DIM>::Q;
  const size_t npop = (size_t)(NP + 2) * Q * nc, naux = (size_t)(NP + DIM + 3) * nc;
  // exact-size heap buffers so that the address sanitizer sees any overrun
  std::vector<R> popA(npop), popB(npop), auxA(naux), auxB(naux);
  std::vector<double> fields((size_t)(NP + 2 + DIM) * nc);
  memcpy(fields.data(), phi, (size_t)NP * nc * 8);
  memcpy(fields.data() + (size_t)NP * nc, T, (size_t)nc * 8);
  size_t off = (size_t)(NP + 1) * nc;
  if (u) {
    memcpy(fields.data() + off, u, (size_t)DIM * nc * 8);
    off += (size_t)DIM * nc;
  }
  if (p) memcpy(fields.data() + off, p, (size_t)nc * 8);
  for (long long c = 0; c < nc; ++c)
    init_cell<DIM, NP, R>(P, fields.data(), u ? 1 : 0, p ? 1 : 0, popA.data(), auxA.data(), c);
  for (int s = 0; s < nsteps; ++s) {
    StepArgs<R> a;
    memset(&a, 0, sizeof a);
    a.pin = popA.data();
    a.pout = popB.data();
    a.ain = auxA.data();
    a.aout = auxB.data();
    // poison the outputs: every value must be written by the step
    std::fill(popB.begin(), popB.end(), R(NAN));
    std::fill(auxB.begin(), auxB.end(), R(NAN));
    emulate_step<C, false>(a, P);
    popA.swap(popB);
    auxA.swap(auxB);
  }
  if (pop_out)
    for (size_t k = 0; k < npop; ++k) pop_out[k] = double(popA[k]);
  if (aux_out)
    for (size_t k = 0; k < naux; ++k) aux_out[k] = double(auxA[k]);
  if (mom_out) {
    const int nf = NP + 6 + DIM;
    std::vector<double> plane(nc);
    for (int k = 0; k < nf; ++k) {
      StepArgs<R> a;
      memset(&a, 0, sizeof a);
      a.pin = popA.data();
      a.ain = auxA.data();
      a.aout = auxB.data();  // scratch for the moments pass
      a.mout = plane.data();
      a.mfield = k;
      std::fill(plane.begin(), plane.end(), NAN);
      emulate_step<C, true>(a, P);
      memcpy(mom_out + (size_t)k * nc, plane.data(), (size_t)nc * 8);
    }
  }
  return 0;
}

template <int DIM, typename R, typename RC>
int run_n(const lbf_params* prm, const double* phi, const double* T, const double* u, const double* p,
          int nsteps, double* po, double* ao, double* mo) {
  switch (prm->nphase) {
    case 1: return run<DIM, 1, R, RC>(prm, phi, T, u, p, nsteps, po, ao, mo);
    case 2: return run<DIM, 2, R, RC>(prm, phi, T, u, p, nsteps, po, ao, mo);
    case 3: return run<DIM, 3, R, RC>(prm, phi, T, u, p, nsteps, po, ao, mo);
    case 4: return run<DIM, 4, R, RC>(prm, phi, T, u, p, nsteps, po, ao, mo);
  }
  return -1;
}

}  // namespace

extern "C" int lbf_emu_run(const lbf_params* prm, const double* phi, const double* T, const double* u,
                           const double* p, int nsteps, double* pop_out, double* aux_out,
                           double* mom_out) {
  if (!check_params(prm).empty()) return -1;
  lbf_params q = *prm;
  if (q.dim == 2) q.nz = 1;
  const int d = q.dim, pr = q.precision;
  if (d == 2 && pr == LBF_FP64) return run_n<2, double, double>(&q, phi, T, u, p, nsteps, pop_out, aux_out, mom_out);
  if (d == 2 && pr == LBF_MIXED) return run_n<2, float, double>(&q, phi, T, u, p, nsteps, pop_out, aux_out, mom_out);
  if (d == 2) return run_n<2, float, float>(&q, phi, T, u, p, nsteps, pop_out, aux_out, mom_out);
  if (pr == LBF_FP64) return run_n<3, double, double>(&q, phi, T, u, p, nsteps, pop_out, aux_out, mom_out);
  if (pr == LBF_MIXED) return run_n<3, float, double>(&q, phi, T, u, p, nsteps, pop_out, aux_out, mom_out);
  return run_n<3, float, float>(&q, phi, T, u, p, nsteps, pop_out, aux_out, mom_out);
}

#ifdef LBF_EMU_MAIN
// Sanitizer driver: every lattice, phase count, precision and face
// combination on ragged grids, a few steps each, from a droplet-like start
// with random velocity.  Exit status 0 when every value stays finite.
int main() {
  int bad = 0, runs = 0;
  for (int dim = 2; dim <= 3; ++dim)
    for (int N = 1; N <= 4; ++N)
      for (int prec = 0; prec < 3; ++prec)
        for (int bcase = 0; bcase < 3; ++bcase) {
          lbf_params P;
          memset(&P, 0, sizeof P);
          P.dim = dim;
          P.nx = dim == 2 ? 37 : 33;
          P.ny = dim == 2 ? 11 : 9;
          P.nz = dim == 2 ? 1 : 6;
          P.nphase = N;
          P.precision = prec;
          P.flow_bc[0] = LBF_BC_WALL;
          P.flow_bc[1] = bcase == 1 ? LBF_BC_OPEN : LBF_BC_WALL;
          P.therm_bc[0] = LBF_TBC_DIRICHLET;
          P.therm_bc[1] = bcase == 2 ? LBF_TBC_DIRICHLET : LBF_TBC_ADIABATIC;
          P.T_face[0] = -1;
          P.T_face[1] = 1;
          for (int p = 0; p < N; ++p) {
            const bool fr = (p % 2) == 0;
            P.rho_l[p] = fr ? 1.0 : 0.01 * (p + 1);
            P.rho_s[p] = fr ? 0.9 + 0.1 * p : P.rho_l[p];
            P.mu_l[p] = 0.1 * P.rho_l[p];
            P.mu_s[p] = 0.1 * P.rho_s[p];
            P.lam_l[p] = P.lam_s[p] = 0.1;
            P.cp_l[p] = P.cp_s[p] = 1.0 / P.rho_l[p];
            if (fr) P.cp_s[p] = 1.0;
            if (fr) P.cp_l[p] = 1.0;
            P.latent[p] = fr ? 10.0 : 0.0;
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
          P.gravity[0] = 1e-6;
          std::string e = check_params(&P);
          if (!e.empty()) {
            printf("params rejected: %s\n", e.c_str());
            return 2;
          }
          const long long nc = (long long)P.nx * P.ny * P.nz;
          std::vector<double> phi((size_t)N * nc), T(nc), u((size_t)dim * nc), pr(nc);
          for (long long c = 0; c < nc; ++c) {
            const int x = c % P.nx, y = (c / P.nx) % P.ny, z = c / ((long long)P.nx * P.ny);
            const double wn = dim == 2 ? y : z;
            const double r = sqrt((x - 18.0) * (x - 18.0) + wn * wn + (dim == 3 ? (y - 5.0) * (y - 5.0) : 0.0));
            const double d = 0.5 + 0.5 * tanh((8.0 - r) / 2.0);
            double rest = 1.0;
            for (int p = 0; p < N; ++p) {
              const double v = (p == N - 1) ? rest : rest * (p == 0 ? d : 0.5);
              phi[(size_t)p * nc + c] = v;
              rest -= v;
            }
            T[c] = 0.05 * sin(0.7 * x + 0.3 * y);
            for (int a = 0; a < dim; ++a) u[(size_t)a * nc + c] = 1e-3 * cos(0.5 * x + a);
            pr[c] = 1e-4 * sin(0.2 * x);
          }
          const size_t npop = (size_t)(N + 2) * (dim == 2 ? 9 : 19) * nc, naux = (size_t)(N + dim + 3) * nc;
          std::vector<double> po(npop), ao(naux), mo((size_t)(N + 6 + dim) * nc);
          lbf_emu_run(&P, phi.data(), T.data(), u.data(), pr.data(), 3, po.data(), ao.data(), mo.data());
          ++runs;
          bool ok = true;
          for (double v : po) ok = ok && isfinite(v);
          for (double v : ao) ok = ok && isfinite(v);
          for (double v : mo) ok = ok && isfinite(v);
          if (!ok) {
            printf("non-finite output: dim=%d N=%d prec=%d bc=%d\n", dim, N, prec, bcase);
            ++bad;
          }
        }
  printf("%d runs, %d with non-finite output\n", runs, bad);
  return bad ? 1 : 0;
}
#endif
