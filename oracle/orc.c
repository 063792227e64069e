/*
 * Plain FP64 CPU oracle of the coupled lattice-Boltzmann (LB) freezing step
 * of Huang, Zhan, Chai, Huang and Liu, "A diffuse-interface model for N-phase
 * flows with liquid-solid phase change" (arXiv:2603.22902).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
 * HIP library.  It may be loaded by the test suite, by the package's smoke
 * check and by the CPU-baseline leg of the benchmark, and by nothing else.
 * It shares no code, header, table or constant with the GPU path.
 *
 * The step is written cell by cell in the order of the paper's Sec. 3, with
 * no blocking or fusion:
 *   1. zeroth moments of g_{i,p} and h_i (Sec. 3, order-parameter and
 *      total-enthalpy moments) with the lagged divergence source;
 *   2. enthalpy inversion, eq. (H), with mixture thresholds built from
 *      eq. (eq2);
 *   3. isotropic finite differences of phi_p, rho and f_s*phi_p;
 *   4. interface physics of Sec. 2: pairwise normals, R_p, the chemical
 *      potential mu_p and the surface force F_s = sum_p mu_p grad phi_p;
 *   5. flow macros of Sec. 3 (u*, the solid penalty f, u, p) and the
 *      volume-change source mdot of eq. (fluid2);
 *   6. BGK collision of the three LBs with their forcing/source terms;
 *   7. streaming with the boundary rules, storing the lagged fields.
 * Where the paper is silent or garbled the reading taken is stated at the
 * point of use.
 *
 * Lattice units: dx = dt = 1, c_s^2 = 1/3.  Sums over directions run in
 * index order, sums over phases and pairs in ascending order.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OMAXP 4
#define OMAXQ 19

enum { O_WALL = 0, O_OPEN = 1 };
enum { O_DIRICHLET = 0, O_ADIABATIC = 1 };

/* Physical and numerical parameters, all in lattice units. */
typedef struct {
  int dim, nx, ny, nz, nphase;
  int flow_bc[2];   /* wall-normal faces (lo, hi): O_WALL or O_OPEN        */
  int therm_bc[2];  /* wall-normal faces (lo, hi): O_DIRICHLET/O_ADIABATIC */
  double T_face[2]; /* face temperature for Dirichlet faces               */
  double rho_l[OMAXP], rho_s[OMAXP], mu_l[OMAXP], mu_s[OMAXP];
  double lam_l[OMAXP], lam_s[OMAXP], cp_l[OMAXP], cp_s[OMAXP];
  double latent[OMAXP];
  int freezes[OMAXP];
  double sigma[OMAXP][OMAXP];
  double cos_theta[OMAXP][OMAXP]; /* wetting at the lo wall, antisymmetric */
  double eps, tau_g, T_melt, E_ref;
  double gravity[3];
} orc_params;

typedef struct {
  int Q;
  int c[OMAXQ][3];
  double w[OMAXQ];
  int opp[OMAXQ];
} lattice;

/* Macroscopic values of one cell at the current time level. */
typedef struct {
  double phi[OMAXP];
  double rhoH, T, fl, fs, psi, rho, mu, lam, cp;
} cellmac;

typedef struct {
  orc_params P;
  lattice L;
  int N, Q, dim, wn;  /* wn: wall-normal axis (y in 2D, z in 3D) */
  int n[3];
  long ncell, narea;  /* narea: cells of one wall-normal layer      */
  int nlat;           /* number of lattices: f, g_1..g_N, h          */
  double *pop;        /* post-stream populations [lat*Q+i][cell]     */
  double *post;       /* post-collision populations [lat*Q+i][cell]  */
  double *bcin;       /* incoming values on boundary links [face][lat*Q+i][area] */
  double *aux, *aux_new; /* lagged fields [k][cell], see AUX_* below */
  cellmac *mac;
  double *out_u, *out_p, *out_mdot; /* flow macros of the last pass */
  long step;
  int div_mode;  /* ORC_DIV_*: what div u means in G_{i,p}, H_i and the moments */
  int mdot_mode; /* ORC_MDOT_*: which terms of eq. (fluid2) form mdot        */
} orc_state;

/* Readings of two passages the paper leaves open, selectable so that the
 * tests can run each of them.
 *   ORC_DIV_MDOT:   div u := mdot, the continuity law eq. (fluid2).
 *   ORC_DIV_LAGGED: the central difference of the previous step's u.
 *   ORC_MDOT_FREEZE:  mdot = -(1/rho) sum_p (rho_p^s - rho_p^l) D(f_s phi_p)/Dt.
 *   ORC_MDOT_PRINTED: the printed eq. (fluid2), which also carries
 *                     -(1/rho) sum_p rho_p^l D phi_p/Dt. */
enum { ORC_DIV_MDOT = 0, ORC_DIV_LAGGED = 1 };
enum { ORC_MDOT_FREEZE = 0, ORC_MDOT_PRINTED = 1 };

/* Lagged-field planes: phi_p^{n-1} (N), f_s^{n-1}, u^{n-1} (dim),
 * D^{n-1} (the velocity divergence used by the sources of step n-1), and
 * q^{n-1} = (rho C_p T D)^{n-1}. */
#define AUX_PHI(p) (p)
#define AUX_FS(N) (N)
#define AUX_U(N, a) ((N) + 1 + (a))
#define AUX_DIV(N, d) ((N) + 1 + (d))
#define AUX_Q(N, d) ((N) + 2 + (d))
#define NAUX(N, d) ((N) + 3 + (d))

/* ------------------------------------------------------------------ */
/* Lattices.  D2Q9 (used for the paper's 2D cases) and D3Q19, BGK.    */
/* ------------------------------------------------------------------ */
static void make_lattice(int dim, lattice *L) {
  memset(L, 0, sizeof(*L));
  if (dim == 2) {
    static const int c2[9][2] = {{0, 0}, {1, 0},  {0, 1},   {-1, 0}, {0, -1},
                                 {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    L->Q = 9;
    for (int i = 0; i < 9; ++i) {
      L->c[i][0] = c2[i][0];
      L->c[i][1] = c2[i][1];
      L->c[i][2] = 0;
      L->w[i] = (i == 0) ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  } else {
    static const int c3[19][3] = {
        {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
        {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
        {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    L->Q = 19;
    for (int i = 0; i < 19; ++i) {
      for (int a = 0; a < 3; ++a) L->c[i][a] = c3[i][a];
      L->w[i] = (i == 0) ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
  }
  for (int i = 0; i < L->Q; ++i)
    for (int j = 0; j < L->Q; ++j)
      if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] &&
          L->c[j][2] == -L->c[i][2])
        L->opp[i] = j;
}

/* ------------------------------------------------------------------ */
/* Mixture law, eq. (eq2): xi = sum_p [f_s phi_p xi_p^s + (1-f_s) phi_p xi_p^l]. */
/* ------------------------------------------------------------------ */
static double mixture(int N, const double *phi, double fs, const double *xs,
                      const double *xl) {
  double x = 0.0;
  for (int p = 0; p < N; ++p) x += fs * phi[p] * xs[p] + (1.0 - fs) * phi[p] * xl[p];
  return x;
}

/* ------------------------------------------------------------------ */
/* Enthalpy inversion, eq. (H).  The paper states it for one material with */
/* solid/liquid densities rho_s, rho_l and enthalpies H_s, H_l.  For a     */
/* mixture cell the solid and liquid states are the eq. (eq2) mixtures     */
/* at f_s = 1 and f_s = 0, the volumetric latent heat is                   */
/* Lv = sum_p phi_p rho_p^l L_p, and solidus = liquidus = T_melt.          */
/* A cell with Lv = 0 and equal thresholds takes f_l = 1 in the (empty)    */
/* mushy branch.                                                           */
/* ------------------------------------------------------------------ */
static void invert(const orc_params *P, const double *phi, double rhoH, double *T,
                   double *fl) {
  int N = P->nphase;
  double rs = 0, rl = 0, cs = 0, cl = 0, Lv = 0;
  for (int p = 0; p < N; ++p) {
    rs += phi[p] * P->rho_s[p];
    rl += phi[p] * P->rho_l[p];
    cs += phi[p] * P->cp_s[p];
    cl += phi[p] * P->cp_l[p];
    Lv += phi[p] * P->rho_l[p] * P->latent[p];
  }
  double Tm = P->T_melt;
  double Es = rs * cs * Tm;       /* rho_s H_s */
  double El = rl * cl * Tm + Lv;  /* rho_l H_l */
  if (rhoH < Es) {
    *fl = 0.0;
    *T = rhoH / (rs * cs);
  } else if (rhoH > El) {
    *fl = 1.0;
    *T = Tm + (rhoH - El) / (rl * cl);
  } else {
    *fl = (El > Es) ? (rhoH - Es) / (El - Es) : 1.0;
    *T = Tm; /* T_s + f_l (T_l - T_s) with T_s = T_l = T_melt */
  }
}

/* Forward map (T, f_l) -> rho H consistent with invert(). */
static double enthalpy(const orc_params *P, const double *phi, double T, double fl) {
  int N = P->nphase;
  double rs = 0, rl = 0, cs = 0, cl = 0, Lv = 0;
  for (int p = 0; p < N; ++p) {
    rs += phi[p] * P->rho_s[p];
    rl += phi[p] * P->rho_l[p];
    cs += phi[p] * P->cp_s[p];
    cl += phi[p] * P->cp_l[p];
    Lv += phi[p] * P->rho_l[p] * P->latent[p];
  }
  double Es = rs * cs * P->T_melt, El = rl * cl * P->T_melt + Lv;
  if (fl <= 0.0) return rs * cs * T;
  if (fl >= 1.0) return rl * cl * T + Lv;
  return Es + fl * (El - Es);
}

static void cell_props(const orc_params *P, cellmac *m) {
  int N = P->nphase;
  m->fs = 1.0 - m->fl;
  m->psi = 0.0;
  for (int p = 0; p < N; ++p)
    if (P->freezes[p]) m->psi += m->phi[p];
  m->rho = mixture(N, m->phi, m->fs, P->rho_s, P->rho_l);
  m->mu = mixture(N, m->phi, m->fs, P->mu_s, P->mu_l);
  m->lam = mixture(N, m->phi, m->fs, P->lam_s, P->lam_l);
  m->cp = mixture(N, m->phi, m->fs, P->cp_s, P->cp_l);
}

/* ------------------------------------------------------------------ */
/* Equilibria and source terms (Sec. 3).                               */
/* ------------------------------------------------------------------ */
static double cdotu(const lattice *L, int i, const double *u) {
  return L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
}

/* s_i(u) = w_i [c.u/cs2 + (c.u)^2/(2 cs4) - u.u/(2 cs2)] */
static double s_i(const lattice *L, int i, const double *u) {
  double cu = cdotu(L, i, u), uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return L->w[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

/* Pressure-based flow equilibrium: i = 0: p/cs2 (w_0 - 1) + rho s_0;
 * i != 0: p/cs2 w_i + rho s_i. */
static double feq_i(const lattice *L, int i, double p, double rho, const double *u) {
  if (i == 0) return 3.0 * p * (L->w[0] - 1.0) + rho * s_i(L, 0, u);
  return 3.0 * p * L->w[i] + rho * s_i(L, i, u);
}

/* Phase-field equilibrium w_i phi (1 + c.u/cs2). */
static double geq_i(const lattice *L, int i, double phi, const double *u) {
  return L->w[i] * phi * (1.0 + 3.0 * cdotu(L, i, u));
}

/* Total-enthalpy equilibrium.  The paper writes the rest-population trick
 * with rho C_p T (C_p,ref / C_p); this oracle reads the factor as
 * E_ref / (rho C_p) with the constant E_ref = rho_ref C_p,ref, which makes
 * the second moment c_s^2 E_ref T I and, with tau_h = lambda/(E_ref cs2) + 1/2,
 * recovers div(lambda grad T) of eq. (eq4). */
static double heq_i(const lattice *L, int i, double rhoH, double T, double rhocp,
                    double Eref, const double *u) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  if (i == 0) return rhoH - Eref * T + L->w[0] * (Eref * T - 1.5 * rhocp * T * uu);
  double cu = cdotu(L, i, u);
  return L->w[i] * (Eref * T + rhocp * T * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
}

/* Flow forcing F_i = w_i [S + c_i.(F + rho a)/cs2 + (c_i c_i - cs2 I):Lambda/(2 cs4)]
 * with Lambda = uF + Fu + (2/d) rho cs2 S I.  The paper adds the penalty
 * "f" (an acceleration) to the force density F; it is taken as the force
 * density rho a. */
static double force_i(const lattice *L, int dim, int i, double S, const double *F,
                      const double *rhoa, const double *u, double rho) {
  double Lam[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Lam[a][b] = u[a] * F[b] + F[a] * u[b] +
                  ((a == b && a < dim) ? (2.0 / dim) * rho * (1.0 / 3.0) * S : 0.0);
  double cF = 0.0;
  for (int a = 0; a < dim; ++a) cF += L->c[i][a] * (F[a] + rhoa[a]);
  double q = 0.0;
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b)
      q += (L->c[i][a] * L->c[i][b] - (a == b ? 1.0 / 3.0 : 0.0)) * Lam[a][b];
  return L->w[i] * (S + 3.0 * cF + 4.5 * q);
}

/* ------------------------------------------------------------------ */
/* Interface physics of Sec. 2.                                        */
/* ------------------------------------------------------------------ */
static double gprime(double x) { return 2.0 * x * (1.0 - x) * (1.0 - 2.0 * x); }

/* Pairwise normal n_pq = grad phi_pq / |grad phi_pq| with
 * phi_pq = phi_p / (phi_p + phi_q).  By the quotient rule grad phi_pq is a
 * positive multiple of v = phi_q grad phi_p - phi_p grad phi_q; the norm is
 * regularised as sqrt(v.v + 1e-24) so that the 0/0 limit is 0.  Each pair is
 * computed once (p < q) and n_qp = -n_pq. */
static void interface_terms(const orc_params *P, int dim, const double *phi,
                            const double grad[][3], const double *lap,
                            double R[][3], double *mu, double *Fs) {
  int N = P->nphase;
  double n[OMAXP][OMAXP][3];
  for (int p = 0; p < N; ++p)
    for (int q = p + 1; q < N; ++q) {
      double v[3] = {0, 0, 0}, vv = 0.0;
      for (int a = 0; a < dim; ++a) {
        v[a] = phi[q] * grad[p][a] - phi[p] * grad[q][a];
        vv += v[a] * v[a];
      }
      double inv = 1.0 / sqrt(vv + 1e-24);
      for (int a = 0; a < 3; ++a) {
        n[p][q][a] = v[a] * inv;
        n[q][p][a] = -n[p][q][a];
      }
    }
  /* R_p = sum_{q != p} 4 phi_p phi_q / eps n_pq */
  for (int p = 0; p < N; ++p) {
    for (int a = 0; a < 3; ++a) R[p][a] = 0.0;
    for (int q = 0; q < N; ++q) {
      if (q == p) continue;
      double s = 4.0 * phi[p] * phi[q] / P->eps;
      for (int a = 0; a < dim; ++a) R[p][a] += s * n[p][q][a];
    }
  }
  /* mu_p = sum_{q!=p} 2 beta_pq [g'(phi_p) - g'(phi_p+phi_q)] - sum_{q!=p} k_pq lap phi_q,
   * beta_pq = 3 sigma_pq / eps, k_pq = -3 eps sigma_pq / 4, g = phi^2 (1-phi)^2. */
  for (int p = 0; p < N; ++p) {
    double bulk = 0.0, grad_term = 0.0;
    for (int q = 0; q < N; ++q) {
      if (q == p) continue;
      double beta = 3.0 * P->sigma[p][q] / P->eps;
      bulk += 2.0 * beta * (gprime(phi[p]) - gprime(phi[p] + phi[q]));
    }
    for (int q = 0; q < N; ++q) {
      if (q == p) continue;
      double k = -0.75 * P->eps * P->sigma[p][q];
      grad_term += k * lap[q];
    }
    mu[p] = bulk - grad_term;
  }
  /* F_s = sum_p mu_p grad phi_p */
  for (int a = 0; a < 3; ++a) Fs[a] = 0.0;
  for (int p = 0; p < N; ++p)
    for (int a = 0; a < dim; ++a) Fs[a] += mu[p] * grad[p][a];
}

/* Isotropic central stencils: grad X = (1/cs2) sum_i w_i c_i X(x+c_i),
 * lap X = (2/cs2) sum_i w_i [X(x+c_i) - X(x)].  Xn[i] holds X(x+c_i). */
static void stencil(const lattice *L, int dim, const double *Xn, double *grad,
                    double *lap) {
  for (int a = 0; a < 3; ++a) grad[a] = 0.0;
  double l = 0.0;
  for (int i = 0; i < L->Q; ++i) {
    for (int a = 0; a < dim; ++a) grad[a] += L->w[i] * L->c[i][a] * Xn[i];
    l += L->w[i] * (Xn[i] - Xn[0]);
  }
  for (int a = 0; a < dim; ++a) grad[a] *= 3.0;
  if (lap) *lap = 6.0 * l;
}

/* ------------------------------------------------------------------ */
/* Grid helpers.                                                       */
/* ------------------------------------------------------------------ */
static long cell_index(const orc_state *st, const int *x) {
  return ((long)x[2] * st->n[1] + x[1]) * st->n[0] + x[0];
}
static void cell_coords(const orc_state *st, long c, int *x) {
  x[0] = (int)(c % st->n[0]);
  x[1] = (int)((c / st->n[0]) % st->n[1]);
  x[2] = (int)(c / ((long)st->n[0] * st->n[1]));
}
/* Index of the cell within its wall-normal layer. */
static long area_index(const orc_state *st, const int *x) {
  return (st->dim == 2) ? x[0] : (long)x[1] * st->n[0] + x[0];
}
/* y = x + s*c_i with periodic wrap on the lateral axes.  Returns the face
 * (0 = lo, 1 = hi) when the wall-normal coordinate leaves the domain, else -1. */
static int shift(const orc_state *st, const int *x, int i, int s, int *y) {
  int face = -1;
  for (int a = 0; a < 3; ++a) {
    int v = x[a] + s * st->L.c[i][a];
    if (a == st->wn) {
      if (v < 0) face = 0;
      else if (v >= st->n[a]) face = 1;
    } else {
      v = ((v % st->n[a]) + st->n[a]) % st->n[a];
    }
    y[a] = v;
  }
  return face;
}

#define POP(arr, l, i, c) (arr)[((long)(l) * st->Q + (i)) * st->ncell + (c)]

/* ------------------------------------------------------------------ */
/* Step 1-2: moments and inversion of one cell.                        */
/* ------------------------------------------------------------------ */
/* phi_p = sum_i g_{i,p} + (dt/2) phi_p div u is solved for phi_p with the
 * divergence D^{n-1} that the previous step's sources used.  The enthalpy
 * moment is printed as sum h_i + (dt/2) rho C_p T u, which adds a vector to
 * a scalar; it is read as the zeroth-moment correction
 * (dt/2) (rho C_p T D)^{n-1} that matches the source H_i. */
static void cell_macros(const orc_state *st, long c, cellmac *m) {
  int N = st->N, Q = st->Q, d = st->dim;
  double div_prev = st->aux[(long)AUX_DIV(N, d) * st->ncell + c];
  double q_prev = st->aux[(long)AUX_Q(N, d) * st->ncell + c];
  for (int p = 0; p < N; ++p) {
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += POP(st->pop, 1 + p, i, c);
    m->phi[p] = s / (1.0 - 0.5 * div_prev);
  }
  double sh = 0.0;
  for (int i = 0; i < Q; ++i) sh += POP(st->pop, N + 1, i, c);
  m->rhoH = sh + 0.5 * q_prev;
  invert(&st->P, m->phi, m->rhoH, &m->T, &m->fl);
  cell_props(&st->P, m);
}

/* ------------------------------------------------------------------ */
/* Finite-difference inputs at the neighbours of a cell.              */
/* Outside the wall-normal range a ghost layer is used.  At the lo face */
/* of a wall the order parameters follow the geometric wetting rule     */
/* phi_p(ghost) = phi_p + (4/eps) sum_{q!=p} phi_p phi_q cos(theta_pq),  */
/* evaluated with the values of the boundary cell next to the ghost (a   */
/* contact angle of 90 degrees gives a plain copy).  Elsewhere, and for  */
/* f_s and rho, the ghost copies the boundary cell.                      */
/* ------------------------------------------------------------------ */
typedef struct {
  double phi[OMAXP], fs, rho;
} fdval;

static void neighbour_values(const orc_state *st, const int *x, int i, fdval *v) {
  int y[3];
  int face = shift(st, x, i, +1, y);
  int N = st->N;
  if (face < 0) {
    const cellmac *m = &st->mac[cell_index(st, y)];
    for (int p = 0; p < N; ++p) v->phi[p] = m->phi[p];
    v->fs = m->fs;
    v->rho = m->rho;
    return;
  }
  y[st->wn] = (face == 0) ? 0 : st->n[st->wn] - 1;
  const cellmac *b = &st->mac[cell_index(st, y)];
  v->fs = b->fs;
  v->rho = b->rho;
  if (face == 0 && st->P.flow_bc[0] == O_WALL) {
    for (int p = 0; p < N; ++p) {
      double s = 0.0;
      for (int q = 0; q < N; ++q)
        if (q != p) s += b->phi[p] * b->phi[q] * st->P.cos_theta[p][q];
      v->phi[p] = b->phi[p] + 4.0 / st->P.eps * s;
    }
  } else {
    for (int p = 0; p < N; ++p) v->phi[p] = b->phi[p];
  }
}

/* ------------------------------------------------------------------ */
/* Steps 3-6 for one cell.  With store != 0 the post-collision          */
/* populations, the boundary-link values and the new lagged fields are  */
/* written; the flow macros u, p and mdot are always written.           */
/* ------------------------------------------------------------------ */
static void update_cell(orc_state *st, long c, int store) {
  const orc_params *P = &st->P;
  const lattice *L = &st->L;
  int N = st->N, Q = st->Q, d = st->dim;
  const cellmac *m = &st->mac[c];
  int x[3];
  cell_coords(st, c, x);

  /* Step 3: finite differences at time n. */
  fdval nb[OMAXQ];
  for (int i = 0; i < Q; ++i) neighbour_values(st, x, i, &nb[i]);
  double Xn[OMAXQ] = {0};
  double gphi[OMAXP][3], lphi[OMAXP], grho[3], gfsphi[OMAXP][3];
  for (int p = 0; p < N; ++p) {
    for (int i = 0; i < Q; ++i) Xn[i] = nb[i].phi[p];
    stencil(L, d, Xn, gphi[p], &lphi[p]);
  }
  for (int i = 0; i < Q; ++i) Xn[i] = nb[i].rho;
  stencil(L, d, Xn, grho, NULL);
  for (int p = 0; p < N; ++p) {
    for (int a = 0; a < 3; ++a) gfsphi[p][a] = 0.0;
    if (!P->freezes[p]) continue;
    for (int i = 0; i < Q; ++i) Xn[i] = nb[i].fs * nb[i].phi[p];
    stencil(L, d, Xn, gfsphi[p], NULL);
  }

  /* The lagged-difference reading of div u (ORC_DIV_LAGGED): the central
   * difference of the previous step's velocity field u^{n-1}.  Ghost
   * velocities mirror the boundary cell at walls (zero velocity on the face)
   * and copy it at open faces. */
  double Ddiv = 0.0;
  if (st->div_mode == ORC_DIV_LAGGED) {
    const double *aux = st->aux;
    long nc = st->ncell;
    double ug[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      int y[3];
      int face = shift(st, x, i, +1, y);
      double sgn = 1.0;
      if (face >= 0) {
        y[st->wn] = (face == 0) ? 0 : st->n[st->wn] - 1;
        if (P->flow_bc[face] == O_WALL) sgn = -1.0;
      }
      long cy = cell_index(st, y);
      for (int a = 0; a < d; ++a)
        ug[a] += L->w[i] * L->c[i][a] * (sgn * aux[(long)AUX_U(N, a) * nc + cy]);
    }
    for (int a = 0; a < d; ++a) Ddiv += 3.0 * ug[a];
  }

  /* Step 4: interface physics. */
  double R[OMAXP][3], mu[OMAXP], Fs[3];
  interface_terms(P, d, m->phi, (const double(*)[3])gphi, lphi, R, mu, Fs);
  double F[3];
  for (int a = 0; a < 3; ++a) F[a] = Fs[a] + (a < d ? m->rho * P->gravity[a] : 0.0);

  /* Step 5: flow macros.  rho u* = sum c_i f_i + F/2; the penalty
   * f = f_s (u_s - u*) acts only on the frozen part of the freezing phases,
   * so its weight is w_s = f_s * sum_{p freezing} phi_p, with a solid at
   * rest (u_s = 0); u = u* + f/2. */
  double mom[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    double fi = POP(st->pop, 0, i, c);
    for (int a = 0; a < d; ++a) mom[a] += L->c[i][a] * fi;
  }
  double ustar[3] = {0, 0, 0}, acc[3] = {0, 0, 0}, u[3] = {0, 0, 0}, rhoa[3] = {0, 0, 0};
  double ws = m->fs * m->psi;
  for (int a = 0; a < d; ++a) {
    ustar[a] = (mom[a] + 0.5 * F[a]) / m->rho;
    acc[a] = ws * (0.0 - ustar[a]);
    u[a] = ustar[a] + 0.5 * acc[a];
    rhoa[a] = m->rho * acc[a];
  }
  /* Volume source of eq. (fluid2), with D X/Dt = (X^n - X^{n-1})/dt +
   * u^n . grad X^n.  Sec. 2 states that without phase change the flow is
   * divergence free; the freezing term alone gives exactly that when
   * rho_p^s = rho_p^l (ORC_MDOT_FREEZE):
   *   mdot = -(1/rho) sum_p (rho_p^s - rho_p^l) D(f_s phi_p)/Dt.
   * The printed source also carries sum_p rho_p^l D phi_p/Dt, which is not
   * zero inside a diffuse interface even without freezing; ORC_MDOT_PRINTED
   * keeps it. */
  const double *aux = st->aux;
  long nc = st->ncell;
  double fs_prev = aux[(long)AUX_FS(N) * nc + c];
  double msum = 0.0;
  for (int p = 0; p < N; ++p) {
    double phi_prev = aux[(long)AUX_PHI(p) * nc + c];
    double term = 0.0;
    if (P->freezes[p]) {
      double ug = 0.0;
      for (int a = 0; a < d; ++a) ug += u[a] * gfsphi[p][a];
      term += (P->rho_s[p] - P->rho_l[p]) * (m->fs * m->phi[p] - fs_prev * phi_prev + ug);
    }
    if (st->mdot_mode == ORC_MDOT_PRINTED) {
      double ug = 0.0;
      for (int a = 0; a < d; ++a) ug += u[a] * gphi[p][a];
      term += P->rho_l[p] * (m->phi[p] - phi_prev + ug);
    }
    msum += term;
  }
  double mdot = -msum / m->rho;
  /* The continuity reading of div u (ORC_DIV_MDOT): the sources of this
   * step use mdot^n, the moments of the next step mdot^n as their lagged
   * divergence. */
  if (st->div_mode == ORC_DIV_MDOT) Ddiv = mdot;
  /* S = rho mdot + u . grad rho */
  double ugr = 0.0;
  for (int a = 0; a < d; ++a) ugr += u[a] * grho[a];
  double S = m->rho * mdot + ugr;
  double Fi[OMAXQ];
  for (int i = 0; i < Q; ++i) Fi[i] = force_i(L, d, i, S, F, rhoa, u, m->rho);
  double tau_f = 3.0 * m->mu / m->rho + 0.5;
  /* p = cs2/(1-w_0) [sum_{i!=0} f_i + S/2 + (tau_f - 1/2) F_0 + rho s_0(u)] */
  double sf = 0.0;
  for (int i = 1; i < Q; ++i) sf += POP(st->pop, 0, i, c);
  double pr = (1.0 / 3.0) / (1.0 - L->w[0]) *
              (sf + 0.5 * S + (tau_f - 0.5) * Fi[0] + m->rho * s_i(L, 0, u));

  for (int a = 0; a < d; ++a) st->out_u[(long)a * nc + c] = u[a];
  st->out_p[c] = pr;
  st->out_mdot[c] = mdot;
  if (!store) return;

  /* Step 6: collisions. */
  double fe[OMAXQ];
  for (int i = 0; i < Q; ++i) {
    fe[i] = feq_i(L, i, pr, m->rho, u);
    double fi = POP(st->pop, 0, i, c);
    POP(st->post, 0, i, c) = fi - (fi - fe[i]) / tau_f + (1.0 - 0.5 / tau_f) * Fi[i];
  }
  /* Phase field: G = w_i [c_i . d_t(phi u)/cs2 + c_i . R_p] + w_i phi_p div u with
   * d_t(phi u) = phi^n u^n - phi^{n-1} u^{n-1}. */
  double tg = P->tau_g;
  double ge[OMAXP][OMAXQ];
  for (int p = 0; p < N; ++p) {
    double phi_prev = aux[(long)AUX_PHI(p) * nc + c];
    double dphiu[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a)
      dphiu[a] = m->phi[p] * u[a] - phi_prev * aux[(long)AUX_U(N, a) * nc + c];
    for (int i = 0; i < Q; ++i) {
      double cd = 0.0, cr = 0.0;
      for (int a = 0; a < d; ++a) {
        cd += L->c[i][a] * dphiu[a];
        cr += L->c[i][a] * R[p][a];
      }
      double Gi = L->w[i] * (3.0 * cd + cr) + L->w[i] * m->phi[p] * Ddiv;
      ge[p][i] = geq_i(L, i, m->phi[p], u);
      double gi = POP(st->pop, 1 + p, i, c);
      POP(st->post, 1 + p, i, c) = gi - (gi - ge[p][i]) / tg + (1.0 - 0.5 / tg) * Gi;
    }
  }
  /* Enthalpy: H_i = w_i rho C_p T div u (the printed source has no lattice
   * weight; without one its zeroth moment would be Q times too large),
   * tau_h = lambda/(E_ref cs2) + 1/2. */
  double rhocp = m->rho * m->cp;
  double tau_h = 3.0 * m->lam / P->E_ref + 0.5;
  double he[OMAXQ];
  for (int i = 0; i < Q; ++i) {
    he[i] = heq_i(L, i, m->rhoH, m->T, rhocp, P->E_ref, u);
    double Hi = L->w[i] * rhocp * m->T * Ddiv;
    double hi = POP(st->pop, N + 1, i, c);
    POP(st->post, N + 1, i, c) = hi - (hi - he[i]) / tau_h + (1.0 - 0.5 / tau_h) * Hi;
  }

  /* Boundary links: the values that enter this cell at the next step through
   * the wall-normal faces.  Walls: halfway bounce-back for f and g (no slip,
   * no flux); for h, bounce-back at adiabatic walls and non-equilibrium
   * extrapolation at Dirichlet faces, with a ghost node half a cell outside
   * the face at T_g = 2 T_face - T (so the face sits at T_face), the ghost's
   * velocity 0 at walls and u at open faces, and this cell's non-equilibrium
   * part.  Open faces: non-equilibrium extrapolation of f with ghost
   * pressure 0 and this cell's u and rho, of g with this cell's phi and u,
   * and of h as above (T_g = T at adiabatic open faces). */
  for (int face = 0; face < 2; ++face) {
    int edge = (face == 0) ? 0 : st->n[st->wn] - 1;
    if (x[st->wn] != edge) continue;
    int dir = (face == 0) ? +1 : -1; /* c_i component pointing into the domain */
    long ai = area_index(st, x);
    for (int i = 0; i < Q; ++i) {
      if (L->c[i][st->wn] != dir) continue;
      int o = L->opp[i];
      double *bc = st->bcin + (long)face * st->nlat * Q * st->narea;
#define BCIN(l, i) bc[((long)(l) * Q + (i)) * st->narea + ai]
      if (P->flow_bc[face] == O_WALL) {
        BCIN(0, i) = POP(st->post, 0, o, c);
        for (int p = 0; p < N; ++p) BCIN(1 + p, i) = POP(st->post, 1 + p, o, c);
      } else {
        double zero_p = 0.0;
        double fg = feq_i(L, i, zero_p, m->rho, u);
        BCIN(0, i) = fg + (1.0 - 1.0 / tau_f) * (POP(st->pop, 0, i, c) - fe[i]);
        for (int p = 0; p < N; ++p)
          BCIN(1 + p, i) = ge[p][i] + (1.0 - 1.0 / tg) * (POP(st->pop, 1 + p, i, c) - ge[p][i]);
      }
      if (P->flow_bc[face] == O_WALL && P->therm_bc[face] == O_ADIABATIC) {
        BCIN(N + 1, i) = POP(st->post, N + 1, o, c);
      } else {
        double Tg = (P->therm_bc[face] == O_DIRICHLET) ? 2.0 * P->T_face[face] - m->T : m->T;
        double ug[3] = {0, 0, 0};
        if (P->flow_bc[face] == O_OPEN)
          for (int a = 0; a < 3; ++a) ug[a] = u[a];
        double hg = heq_i(L, i, 0.0, Tg, rhocp, P->E_ref, ug); /* i != 0: rhoH unused */
        BCIN(N + 1, i) = hg + (1.0 - 1.0 / tau_h) * (POP(st->pop, N + 1, i, c) - he[i]);
      }
#undef BCIN
    }
  }

  /* Lagged fields for the next step. */
  double *an = st->aux_new;
  for (int p = 0; p < N; ++p) an[(long)AUX_PHI(p) * nc + c] = m->phi[p];
  an[(long)AUX_FS(N) * nc + c] = m->fs;
  for (int a = 0; a < d; ++a) an[(long)AUX_U(N, a) * nc + c] = u[a];
  an[(long)AUX_DIV(N, d) * nc + c] = Ddiv;
  an[(long)AUX_Q(N, d) * nc + c] = rhocp * m->T * Ddiv;
}

/* Step 7: streaming, f_i(x, t+1) = f_i^+(x - c_i, t), boundary links from bcin. */
static void stream(orc_state *st) {
  int Q = st->Q;
  long nc = st->ncell;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < nc; ++c) {
    int x[3], y[3];
    cell_coords(st, c, x);
    long ai = area_index(st, x);
    for (int i = 0; i < Q; ++i) {
      int face = shift(st, x, i, -1, y);
      if (face < 0) {
        long src = cell_index(st, y);
        for (int l = 0; l < st->nlat; ++l) POP(st->pop, l, i, c) = POP(st->post, l, i, src);
      } else {
        const double *bc = st->bcin + (long)face * st->nlat * Q * st->narea;
        for (int l = 0; l < st->nlat; ++l)
          POP(st->pop, l, i, c) = bc[((long)l * Q + i) * st->narea + ai];
      }
    }
  }
}

static void all_macros(orc_state *st) {
#pragma omp parallel for schedule(static)
  for (long c = 0; c < st->ncell; ++c) cell_macros(st, c, &st->mac[c]);
}

/* ================================================================== */
/* Exported interface (ctypes).                                       */
/* ================================================================== */
orc_state *orc_create(const orc_params *P) {
  if (P->dim != 2 && P->dim != 3) return NULL;
  if (P->nphase < 1 || P->nphase > OMAXP) return NULL;
  orc_state *st = (orc_state *)calloc(1, sizeof(orc_state));
  st->P = *P;
  st->dim = P->dim;
  st->N = P->nphase;
  make_lattice(P->dim, &st->L);
  st->Q = st->L.Q;
  st->n[0] = P->nx;
  st->n[1] = P->ny;
  st->n[2] = (P->dim == 2) ? 1 : P->nz;
  st->wn = P->dim - 1;
  st->ncell = (long)st->n[0] * st->n[1] * st->n[2];
  st->narea = st->ncell / st->n[st->wn];
  st->nlat = st->N + 2;
  st->div_mode = ORC_DIV_LAGGED;
  st->mdot_mode = ORC_MDOT_FREEZE;
  long np = (long)st->nlat * st->Q * st->ncell;
  long na = (long)NAUX(st->N, st->dim) * st->ncell;
  st->pop = (double *)calloc(np, sizeof(double));
  st->post = (double *)calloc(np, sizeof(double));
  st->bcin = (double *)calloc((long)2 * st->nlat * st->Q * st->narea, sizeof(double));
  st->aux = (double *)calloc(na, sizeof(double));
  st->aux_new = (double *)calloc(na, sizeof(double));
  st->mac = (cellmac *)calloc(st->ncell, sizeof(cellmac));
  st->out_u = (double *)calloc((long)st->dim * st->ncell, sizeof(double));
  st->out_p = (double *)calloc(st->ncell, sizeof(double));
  st->out_mdot = (double *)calloc(st->ncell, sizeof(double));
  if (!st->pop || !st->post || !st->bcin || !st->aux || !st->aux_new || !st->mac ||
      !st->out_u || !st->out_p || !st->out_mdot) {
    free(st->pop); free(st->post); free(st->bcin); free(st->aux); free(st->aux_new);
    free(st->mac); free(st->out_u); free(st->out_p); free(st->out_mdot);
    free(st);
    return NULL;
  }
  return st;
}

void orc_destroy(orc_state *st) {
  if (!st) return;
  free(st->pop); free(st->post); free(st->bcin); free(st->aux); free(st->aux_new);
  free(st->mac); free(st->out_u); free(st->out_p); free(st->out_mdot);
  free(st);
}

long orc_ncell(const orc_state *st) { return st->ncell; }

/* Select the readings (ORC_DIV_*, ORC_MDOT_*); returns 0, or -1 if either
 * value is unknown (the state is then unchanged). */
int orc_set_readings(orc_state *st, int div_mode, int mdot_mode) {
  if (div_mode != ORC_DIV_MDOT && div_mode != ORC_DIV_LAGGED) return -1;
  if (mdot_mode != ORC_MDOT_FREEZE && mdot_mode != ORC_MDOT_PRINTED) return -1;
  st->div_mode = div_mode;
  st->mdot_mode = mdot_mode;
  return 0;
}
int orc_q(const orc_state *st) { return st->Q; }
int orc_naux(const orc_state *st) { return NAUX(st->N, st->dim); }
long orc_step_count(const orc_state *st) { return st->step; }

/* Initial state: f_l = 1 where T > T_melt else 0, rho H from the forward map,
 * populations at equilibrium, lagged fields (phi^0, f_s^0, u^0, 0, 0).
 * phi: [N][cell], T: [cell], u: [dim][cell] or NULL, p: [cell] or NULL. */
void orc_init(orc_state *st, const double *phi, const double *T, const double *u,
              const double *p) {
  int N = st->N, Q = st->Q, d = st->dim;
  long nc = st->ncell;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < nc; ++c) {
    cellmac m;
    for (int q = 0; q < N; ++q) m.phi[q] = phi[(long)q * nc + c];
    m.T = T[c];
    m.fl = (m.T > st->P.T_melt) ? 1.0 : 0.0;
    m.rhoH = enthalpy(&st->P, m.phi, m.T, m.fl);
    cell_props(&st->P, &m);
    double uc[3] = {0, 0, 0};
    if (u)
      for (int a = 0; a < d; ++a) uc[a] = u[(long)a * nc + c];
    double pc = p ? p[c] : 0.0;
    for (int i = 0; i < Q; ++i) {
      POP(st->pop, 0, i, c) = feq_i(&st->L, i, pc, m.rho, uc);
      for (int q = 0; q < N; ++q) POP(st->pop, 1 + q, i, c) = geq_i(&st->L, i, m.phi[q], uc);
      POP(st->pop, N + 1, i, c) = heq_i(&st->L, i, m.rhoH, m.T, m.rho * m.cp, st->P.E_ref, uc);
    }
    for (int q = 0; q < N; ++q) st->aux[(long)AUX_PHI(q) * nc + c] = m.phi[q];
    st->aux[(long)AUX_FS(N) * nc + c] = m.fs;
    for (int a = 0; a < d; ++a) st->aux[(long)AUX_U(N, a) * nc + c] = uc[a];
    st->aux[(long)AUX_DIV(N, d) * nc + c] = 0.0;
    st->aux[(long)AUX_Q(N, d) * nc + c] = 0.0;
  }
  st->step = 0;
}

void orc_step(orc_state *st, int nsteps) {
  for (int s = 0; s < nsteps; ++s) {
    all_macros(st);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < st->ncell; ++c) update_cell(st, c, 1);
    stream(st);
    double *t = st->aux;
    st->aux = st->aux_new;
    st->aux_new = t;
    st->step++;
  }
}

/* Macroscopic fields at the current time level, each a [cell] plane:
 * phi_p (N planes), rhoH, T, f_l, rho, u (dim planes), p, mdot. */
void orc_moments(orc_state *st, double *out) {
  int N = st->N, d = st->dim;
  long nc = st->ncell;
  all_macros(st);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < nc; ++c) update_cell(st, c, 0);
  long k = 0;
  for (int p = 0; p < N; ++p, ++k)
    for (long c = 0; c < nc; ++c) out[k * nc + c] = st->mac[c].phi[p];
  for (long c = 0; c < nc; ++c) out[k * nc + c] = st->mac[c].rhoH;
  ++k;
  for (long c = 0; c < nc; ++c) out[k * nc + c] = st->mac[c].T;
  ++k;
  for (long c = 0; c < nc; ++c) out[k * nc + c] = st->mac[c].fl;
  ++k;
  for (long c = 0; c < nc; ++c) out[k * nc + c] = st->mac[c].rho;
  ++k;
  for (int a = 0; a < d; ++a, ++k)
    for (long c = 0; c < nc; ++c) out[k * nc + c] = st->out_u[(long)a * nc + c];
  for (long c = 0; c < nc; ++c) out[k * nc + c] = st->out_p[c];
  ++k;
  for (long c = 0; c < nc; ++c) out[k * nc + c] = st->out_mdot[c];
}

/* Conservation diagnostics at the current time level:
 * out = [m_p (N), V_s^p (N), V_sl^p (N), sum rhoH, max |sum_p phi_p - 1|,
 *        front, nonfinite] with m_p = sum phi_p [f_s rho_p^s + (1-f_s) rho_p^l],
 * V_s^p = sum f_s phi_p, V_sl^p = sum phi_p, and the front the
 * volume-equivalent solid thickness sum f_s psi / (cells per wall layer). */
void orc_diagnostics(orc_state *st, double *out) {
  int N = st->N;
  all_macros(st);
  double m[OMAXP] = {0}, vs[OMAXP] = {0}, vsl[OMAXP] = {0}, srh = 0, err = 0, sol = 0;
  double bad = 0;
  for (long c = 0; c < st->ncell; ++c) {
    const cellmac *cm = &st->mac[c];
    double s = 0.0;
    for (int p = 0; p < N; ++p) {
      m[p] += cm->phi[p] * (cm->fs * st->P.rho_s[p] + (1.0 - cm->fs) * st->P.rho_l[p]);
      vs[p] += cm->fs * cm->phi[p];
      vsl[p] += cm->phi[p];
      s += cm->phi[p];
      if (!isfinite(cm->phi[p])) bad = 1;
    }
    if (!isfinite(cm->rhoH)) bad = 1;
    srh += cm->rhoH;
    double e = fabs(s - 1.0);
    if (e > err) err = e;
    sol += cm->fs * cm->psi;
  }
  for (int p = 0; p < N; ++p) {
    out[p] = m[p];
    out[N + p] = vs[p];
    out[2 * N + p] = vsl[p];
  }
  out[3 * N] = srh;
  out[3 * N + 1] = err;
  out[3 * N + 2] = sol / (double)st->narea;
  out[3 * N + 3] = bad;
}

void orc_get_state(const orc_state *st, double *pop, double *aux) {
  long np = (long)st->nlat * st->Q * st->ncell;
  if (pop) memcpy(pop, st->pop, np * sizeof(double));
  if (aux) memcpy(aux, st->aux, (long)NAUX(st->N, st->dim) * st->ncell * sizeof(double));
}

void orc_set_state(orc_state *st, const double *pop, const double *aux) {
  long np = (long)st->nlat * st->Q * st->ncell;
  if (pop) memcpy(st->pop, pop, np * sizeof(double));
  if (aux) memcpy(st->aux, aux, (long)NAUX(st->N, st->dim) * st->ncell * sizeof(double));
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---- single-cell entry points used by the pin tests ---------------- */
int orc_lattice(int dim, int *c, double *w) {
  lattice L;
  make_lattice(dim, &L);
  for (int i = 0; i < L.Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
    w[i] = L.w[i];
  }
  return L.Q;
}
void orc_feq(int dim, double p, double rho, const double *u, double *out) {
  lattice L;
  make_lattice(dim, &L);
  for (int i = 0; i < L.Q; ++i) out[i] = feq_i(&L, i, p, rho, u);
}
void orc_geq(int dim, double phi, const double *u, double *out) {
  lattice L;
  make_lattice(dim, &L);
  for (int i = 0; i < L.Q; ++i) out[i] = geq_i(&L, i, phi, u);
}
void orc_heq(int dim, double rhoH, double T, double rhocp, double Eref, const double *u,
             double *out) {
  lattice L;
  make_lattice(dim, &L);
  for (int i = 0; i < L.Q; ++i) out[i] = heq_i(&L, i, rhoH, T, rhocp, Eref, u);
}
void orc_force(int dim, double S, const double *F, const double *rhoa, const double *u,
               double rho, double *out) {
  lattice L;
  make_lattice(dim, &L);
  for (int i = 0; i < L.Q; ++i) out[i] = force_i(&L, dim, i, S, F, rhoa, u, rho);
}
void orc_stencil(int dim, const double *Xn, double *grad, double *lap) {
  lattice L;
  make_lattice(dim, &L);
  stencil(&L, dim, Xn, grad, lap);
}
void orc_invert(const orc_params *P, const double *phi, double rhoH, double *T, double *fl) {
  invert(P, phi, rhoH, T, fl);
}
double orc_enthalpy(const orc_params *P, const double *phi, double T, double fl) {
  return enthalpy(P, phi, T, fl);
}
void orc_interface(const orc_params *P, const double *phi, const double *grad,
                   const double *lap, double *R, double *mu, double *Fs) {
  double g[OMAXP][3], r[OMAXP][3];
  for (int p = 0; p < P->nphase; ++p)
    for (int a = 0; a < 3; ++a) g[p][a] = grad[3 * p + a];
  interface_terms(P, P->dim, phi, (const double(*)[3])g, lap, r, mu, Fs);
  for (int p = 0; p < P->nphase; ++p)
    for (int a = 0; a < 3; ++a) R[3 * p + a] = r[p][a];
}
/* The step's finite differences applied to an arbitrary scalar field X
 * (copy ghosts at the wall-normal faces): grad [dim][cell], lap [cell]. */
void orc_fd_field(const orc_params *P, const double *X, double *grad, double *lap) {
  orc_state *st = orc_create(P);
  if (!st) return;
  for (long c = 0; c < st->ncell; ++c) {
    for (int p = 0; p < st->N; ++p) st->mac[c].phi[p] = X[c];
    st->mac[c].fs = 0.0;
    st->mac[c].rho = X[c];
  }
  orc_params Pc = *P;
  st->P = Pc;
  st->P.flow_bc[0] = O_OPEN; /* plain copy ghosts */
  for (long c = 0; c < st->ncell; ++c) {
    int x[3];
    cell_coords(st, c, x);
    fdval nb[OMAXQ];
    double Xn[OMAXQ], g[3], l;
    for (int i = 0; i < st->Q; ++i) {
      neighbour_values(st, x, i, &nb[i]);
      Xn[i] = nb[i].rho;
    }
    stencil(&st->L, st->dim, Xn, g, &l);
    for (int a = 0; a < st->dim; ++a) grad[(long)a * st->ncell + c] = g[a];
    lap[c] = l;
  }
  orc_destroy(st);
}
