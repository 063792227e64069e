// Lattice tables and device-side parameter block of the coupled LB step.
//
// D2Q9 and D3Q19 with BGK collisions (Sec. 3 of arXiv:2603.22902 uses the
// single-relaxation form for all three LBs).  The direction order is fixed
// by the library's interface (lbf_get_populations):
//   D2Q9:  rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-)
//   D3Q19: rest, +x, -x, +y, -y, +z, -z, then for the planes xy, xz, yz the
//          pairs (+,+), (-,-), (+,-), (-,+).
// Weights are stored as multiples of 1/36.  The wall-normal axis is y in 2D
// and z in 3D; "lateral" components are the periodic axes.
#pragma once

#include <hip/hip_runtime.h>

namespace lbf {

constexpr int MAXP = 4;

// Blocks of the first diagnostics pass (256 threads each, grid-strided,
// at most DIAG_MAX_BLOCKS): each writes one row of per-block partials.
constexpr int DIAG_MAX_BLOCKS = 1024;
inline int diag_blocks(long long ncell) {
  const long long b = (ncell + 255) / 256;
  return b > DIAG_MAX_BLOCKS ? DIAG_MAX_BLOCKS : (b < 1 ? 1 : (int)b);
}

template <int DIM>
struct Lat;

template <>
struct Lat<2> {
  static constexpr int Q = 9;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int v[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return v[i];
  }
  __host__ __device__ static constexpr int w36(int i) { return i == 0 ? 16 : (i < 5 ? 4 : 1); }
  // lateral (periodic) and wall-normal components
  __host__ __device__ static constexpr int cl0(int i) { return cx(i); }
  __host__ __device__ static constexpr int cl1(int) { return 0; }
  __host__ __device__ static constexpr int cw(int i) { return cy(i); }
  __host__ __device__ static constexpr int c(int i, int a) { return a == 0 ? cx(i) : (a == 1 ? cy(i) : 0); }
};

template <>
struct Lat<3> {
  static constexpr int Q = 19;
  __host__ __device__ static constexpr int cx(int i) {
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
  }
  __host__ __device__ static constexpr int cy(int i) {
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int cz(int i) {
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
  }
  __host__ __device__ static constexpr int opp(int i) {
    constexpr int v[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    return v[i];
  }
  __host__ __device__ static constexpr int w36(int i) { return i == 0 ? 12 : (i < 7 ? 2 : 1); }
  __host__ __device__ static constexpr int cl0(int i) { return cx(i); }
  __host__ __device__ static constexpr int cl1(int i) { return cy(i); }
  __host__ __device__ static constexpr int cw(int i) { return cz(i); }
  __host__ __device__ static constexpr int c(int i, int a) { return a == 0 ? cx(i) : (a == 1 ? cy(i) : cz(i)); }
};

template <typename R, int DIM>
__host__ __device__ constexpr R wgt(int i) {
  return R(Lat<DIM>::w36(i)) / R(36);
}

enum { BC_WALL = 0, BC_OPEN = 1 };
enum { TBC_DIRICHLET = 0, TBC_ADIABATIC = 1 };

// Parameters as the kernels use them; derived coefficients are formed on
// the host once per context.
struct KParams {
  int nx, ny, nz;
  int nwn;              // cells along the wall-normal axis
  long long area;       // cells per wall-normal layer
  long long ncell;
  int flow_bc[2], therm_bc[2];
  int freezes[MAXP];
  double T_face[2];
  double rho_l[MAXP], rho_s[MAXP], mu_l[MAXP], mu_s[MAXP];
  double lam_l[MAXP], lam_s[MAXP], cp_l[MAXP], cp_s[MAXP];
  double latent[MAXP];
  double beta[MAXP][MAXP];  // 3 sigma_pq / eps
  double kpq[MAXP][MAXP];   // -3 eps sigma_pq / 4
  double cth[MAXP][MAXP];   // cos theta_pq at the low wall
  double eps;               // interface width
  double four_eps;          // 4 / eps
  double tau_g, T_melt, E_ref;
  double grav[3];
};

}  // namespace lbf
