/*
 * lc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU reference for one time step of the
 * hybrid lattice-Boltzmann / finite-difference scheme for nematic liquid
 * crystals of Coelho, Araujo and Telo da Gama, "Lattice-Boltzmann simulation
 * of free nematic-isotropic interfaces" (arXiv:1907.13415).  It exists so that
 * the GPU library can be checked against something obviously correct.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it; the GPU library never links, calls or includes it, and the two
 * share no code, headers or tables.
 *
 * Every tensor is handled as a full 3x3 matrix with literal index loops, in
 * the order the paper writes the equations.  No fusion, no blocking.
 *
 * Storage (shared only as an interface convention with the tests):
 *   site index  s = x + nx*(y + ny*z),  periodic in every direction;
 *   populations f[i*N + s], i over the lattice velocities (table below);
 *   order tensor q5[c*N + s], c = (xx, xy, xz, yy, yz); Qzz = -Qxx - Qyy.
 *   parameters p[6] = (A0, gamma, K, Gamma, xi, tau).
 *
 * Readings of the paper used here (where it is silent):
 *   - The collision is BGK with the BGK forcing term printed in Sec. 1.2.1;
 *     lco_run_coll also offers the MRT operator on the standard moment
 *     bases (the paper's operator, whose matrix and rates it does not give).
 *   - The Laplacian is the compact (2d+1)-point second difference summed over
 *     the axes; first derivatives are the central differences of Sec. 1.2.2.
 *   - One step is Jacobi in time: F, rho and u come from the state at step n;
 *     both Heun stages and the collision use that u and F.
 *   - The predictor Q^P is carried as five components with Qzz = -Qxx-Qyy;
 *     the velocity gradient is not recomputed for the corrector.
 *   - F_alpha = d_beta Pi_{alpha beta} (second index), without the
 *     hydrostatic P0 (Sec. 1.2.1).  On the two-dimensional D2Q9 lattice the
 *     z component of F and u is dropped (it has no z velocities).
 *   - A periodic axis of length one has zero central and second differences,
 *     which is how a two-dimensional grid is handled.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define LCO_D2Q9 0
#define LCO_D3Q19 1

/* ---- velocity sets ------------------------------------------------------
 * D2Q9: rest, four axis links, four diagonals.  D3Q19: rest, six axis links,
 * twelve face diagonals.  Weights follow from the Gauss-Hermite quadrature
 * with c_s^2 = 1/3 (Sec. 1.2.1 quotes c_s = 1/sqrt(3)). */
static const int C2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W2[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int C3[19][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W3[19] = {
    1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const double CS2 = 1.0 / 3.0; /* c_s^2, Sec. 1.2.1 */

typedef struct {
  int q;
  const int (*c)[3];
  const double *w;
  int ndim_u; /* velocity components carried by the lattice (2 or 3) */
} lattice_t;

static int get_lattice(int lattice, lattice_t *L) {
  if (lattice == LCO_D2Q9) {
    L->q = 9; L->c = C2; L->w = W2; L->ndim_u = 2;
    return 0;
  }
  if (lattice == LCO_D3Q19) {
    L->q = 19; L->c = C3; L->w = W3; L->ndim_u = 3;
    return 0;
  }
  return -1;
}

/* Host threads of the whole-grid loops (OpenMP): set, and query. */
void lco_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

int lco_threads(void) { return omp_get_max_threads(); }

/* Velocity table export: c[i*3 + a], w[i].  Returns q, or -1. */
int lco_lattice(int lattice, int *c, double *w) {
  lattice_t L;
  if (get_lattice(lattice, &L)) return -1;
  for (int i = 0; i < L.q; i++) {
    for (int a = 0; a < 3; a++) c[i * 3 + a] = L.c[i][a];
    w[i] = L.w[i];
  }
  return L.q;
}

/* ---- grid helpers ------------------------------------------------------- */
typedef struct {
  int nx, ny, nz;
  size_t N;
} grid_t;

static size_t wrap(long v, int n) {
  long r = v % n;
  if (r < 0) r += n;
  return (size_t)r;
}

static size_t site(const grid_t *g, long x, long y, long z) {
  return wrap(x, g->nx) + (size_t)g->nx * (wrap(y, g->ny) + (size_t)g->ny * wrap(z, g->nz));
}

static void coords(const grid_t *g, size_t s, long *x, long *y, long *z) {
  *x = (long)(s % (size_t)g->nx);
  *y = (long)((s / (size_t)g->nx) % (size_t)g->ny);
  *z = (long)(s / ((size_t)g->nx * (size_t)g->ny));
}

/* Neighbour of site s shifted by +/-1 along axis a. */
static size_t shift(const grid_t *g, size_t s, int a, int d) {
  long x, y, z;
  coords(g, s, &x, &y, &z);
  if (a == 0) x += d;
  if (a == 1) y += d;
  if (a == 2) z += d;
  return site(g, x, y, z);
}

/* Site s displaced by the lattice vector c (periodic). */
static size_t displaced(const grid_t *g, size_t s, const int c[3]) {
  long x, y, z;
  coords(g, s, &x, &y, &z);
  return site(g, x + c[0], y + c[1], z + c[2]);
}

/* ---- finite-difference stencils ---------------------------------------------
 * Compact (the default): the central first differences and the (2d+1)-point
 * second difference of Sec. 1.2.2.  Isotropic (lco_set_stencil(1)), the
 * alternative the closing remarks of Sec. 2.2 point to for cutting spurious
 * currents: derivatives from the lattice's own velocity set and weights,
 *   d_g V = (1/cs2) sum_i w_i c_ig V(x + c_i),
 *   lap V = (2/cs2) sum_i w_i [V(x + c_i) - V(x)],
 * exact on linear and quadratic fields, with leading errors that do not
 * depend on the direction.  The mode applies to grad Q, lap Q, the body
 * force and grad u of lco_run_coll, lco_fields and lco_observe (the velocity
 * set is that of the lattice argument); lco_rate and lco_stress are always
 * compact.  `iso` below is that velocity set, or NULL for compact. */
static int g_stencil = 0;

int lco_set_stencil(int mode) {
  if (mode != 0 && mode != 1) return -1;
  g_stencil = mode;
  return 0;
}

int lco_stencil(void) { return g_stencil; }

/* Full symmetric traceless tensor from the five stored components
 * (uniaxial definition and symmetry of Q, Sec. 1.1). */
static void full_Q(const double *q5, size_t N, size_t s, double Q[3][3]) {
  double xx = q5[0 * N + s], xy = q5[1 * N + s], xz = q5[2 * N + s];
  double yy = q5[3 * N + s], yz = q5[4 * N + s];
  Q[0][0] = xx; Q[0][1] = xy; Q[0][2] = xz;
  Q[1][0] = xy; Q[1][1] = yy; Q[1][2] = yz;
  Q[2][0] = xz; Q[2][1] = yz; Q[2][2] = -xx - yy;
}

/* First differences:  dQ[g][a][b] = d_g Q_ab; central (Sec. 1.2.2) or
 * isotropic. */
static void grad_Q(const grid_t *g, const lattice_t *iso, const double *q5, size_t s, double dQ[3][3][3]) {
  if (iso) {
    for (int gg = 0; gg < 3; gg++)
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) dQ[gg][a][b] = 0.0;
    for (int i = 1; i < iso->q; i++) {
      double Qi[3][3];
      full_Q(q5, g->N, displaced(g, s, iso->c[i]), Qi);
      for (int gg = 0; gg < 3; gg++)
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) dQ[gg][a][b] += iso->w[i] * iso->c[i][gg] * Qi[a][b] / CS2;
    }
    return;
  }
  for (int gg = 0; gg < 3; gg++) {
    double Qp[3][3], Qm[3][3];
    full_Q(q5, g->N, shift(g, s, gg, +1), Qp);
    full_Q(q5, g->N, shift(g, s, gg, -1), Qm);
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) dQ[gg][a][b] = (Qp[a][b] - Qm[a][b]) / 2.0;
  }
}

/* Laplacian: compact, the sum over axes of V(x+e) - 2V(x) + V(x-e); or
 * isotropic. */
static void lap_Q(const grid_t *g, const lattice_t *iso, const double *q5, size_t s, double L[3][3]) {
  double Q0[3][3];
  full_Q(q5, g->N, s, Q0);
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) L[a][b] = 0.0;
  if (iso) {
    for (int i = 1; i < iso->q; i++) {
      double Qi[3][3];
      full_Q(q5, g->N, displaced(g, s, iso->c[i]), Qi);
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) L[a][b] += 2.0 * iso->w[i] * (Qi[a][b] - Q0[a][b]) / CS2;
    }
    return;
  }
  for (int gg = 0; gg < 3; gg++) {
    double Qp[3][3], Qm[3][3];
    full_Q(q5, g->N, shift(g, s, gg, +1), Qp);
    full_Q(q5, g->N, shift(g, s, gg, -1), Qm);
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) L[a][b] += Qp[a][b] - 2.0 * Q0[a][b] + Qm[a][b];
  }
}

/* Molecular field, Eq. (4):
 * H = -A0(1-g/3) Q - A0 g (Tr(Q^2) I/3 - Q Q^T) - A0 g Q Tr(Q^2) + K lap Q. */
static void molecular_field(const double Q[3][3], const double L[3][3],
                            const double *p, double H[3][3]) {
  const double A0 = p[0], gam = p[1], K = p[2];
  double trQ2 = 0.0;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) trQ2 += Q[a][b] * Q[a][b];
  for (int a = 0; a < 3; a++) {
    for (int b = 0; b < 3; b++) {
      double QQ = 0.0; /* Q_{a g} Q_{b g} */
      for (int gg = 0; gg < 3; gg++) QQ += Q[a][gg] * Q[b][gg];
      double delta = (a == b) ? 1.0 : 0.0;
      H[a][b] = -A0 * (1.0 - gam / 3.0) * Q[a][b]
                - A0 * gam * (trQ2 * delta / 3.0 - QQ)
                - A0 * gam * Q[a][b] * trQ2
                + K * L[a][b];
    }
  }
}

/* Liquid-crystal stress, Eq. (6), without the hydrostatic -P0 (the body
 * force of Sec. 1.2.1 removes it), with dF/d(d_b Q_gn) = K d_b Q_gn. */
static void stress(const double Q[3][3], const double H[3][3], const double dQ[3][3][3],
                   const double *p, double tau[3][3]) {
  const double K = p[2], xi = p[4];
  double Qp[3][3];
  double QH = 0.0;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      Qp[a][b] = Q[a][b] + ((a == b) ? 1.0 / 3.0 : 0.0);
      QH += Q[a][b] * H[a][b];
    }
  for (int a = 0; a < 3; a++) {
    for (int b = 0; b < 3; b++) {
      double t = 2.0 * xi * Qp[a][b] * QH;
      for (int gg = 0; gg < 3; gg++) t -= xi * H[a][gg] * Qp[gg][b];
      for (int gg = 0; gg < 3; gg++) t -= xi * Qp[a][gg] * H[gg][b];
      for (int gg = 0; gg < 3; gg++)
        for (int n = 0; n < 3; n++) t -= dQ[a][gg][n] * K * dQ[b][gg][n];
      for (int gg = 0; gg < 3; gg++) t += Q[a][gg] * H[gg][b] - H[a][gg] * Q[gg][b];
      tau[a][b] = t;
    }
  }
}

/* Beris-Edwards rate, Eq. (1)-(2): R = Gamma H + S(W, D, Q) - (u . grad) Q,
 * with G[a][b] = d_b u_a, D = (G + G^T)/2, W = (G - G^T)/2. */
static void be_rate(const double Q[3][3], const double H[3][3], const double dQ[3][3][3],
                    const double u[3], const double G[3][3], const double *p,
                    double R[3][3], double Sout[3][3]) {
  const double Gam = p[3], xi = p[4];
  double D[3][3], W[3][3], Qp[3][3];
  double QdU = 0.0; /* Q_{g e} d_g u_e */
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      D[a][b] = (G[a][b] + G[b][a]) / 2.0;
      W[a][b] = (G[a][b] - G[b][a]) / 2.0;
      Qp[a][b] = Q[a][b] + ((a == b) ? 1.0 / 3.0 : 0.0);
    }
  for (int gg = 0; gg < 3; gg++)
    for (int e = 0; e < 3; e++) QdU += Q[gg][e] * G[e][gg];
  for (int a = 0; a < 3; a++) {
    for (int b = 0; b < 3; b++) {
      double S = 0.0;
      for (int gg = 0; gg < 3; gg++) S += (xi * D[a][gg] + W[a][gg]) * Qp[b][gg];
      for (int gg = 0; gg < 3; gg++) S += Qp[a][gg] * (xi * D[gg][b] - W[gg][b]);
      S -= 2.0 * xi * Qp[a][b] * QdU;
      double adv = 0.0;
      for (int gg = 0; gg < 3; gg++) adv += u[gg] * dQ[gg][a][b];
      R[a][b] = Gam * H[a][b] + S - adv;
      if (Sout) Sout[a][b] = S;
    }
  }
}

static void store5(const double T[3][3], double *out5, size_t N, size_t s) {
  out5[0 * N + s] = T[0][0];
  out5[1 * N + s] = T[0][1];
  out5[2 * N + s] = T[0][2];
  out5[3 * N + s] = T[1][1];
  out5[4 * N + s] = T[1][2];
}

/* ---- equilibrium and forcing (Sec. 1.2.1) -------------------------------- */

/* Second-order Hermite equilibrium, Eq. (8). */
static double feq_i(const lattice_t *L, int i, double rho, const double u[3]) {
  double cu = 0.0, uu = 0.0;
  for (int a = 0; a < 3; a++) {
    cu += L->c[i][a] * u[a];
    uu += u[a] * u[a];
  }
  return rho * L->w[i] * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* BGK forcing term S_i printed after Eq. (9). */
static double source_i(const lattice_t *L, int i, double tau, const double u[3], const double F[3]) {
  double cu = 0.0;
  for (int a = 0; a < 3; a++) cu += L->c[i][a] * u[a];
  double s = 0.0;
  for (int a = 0; a < 3; a++) {
    double v = L->c[i][a] / CS2 * (1.0 + cu / CS2) - u[a] / CS2;
    s += v * F[a];
  }
  return L->w[i] * (1.0 - 1.0 / (2.0 * tau)) * s;
}

void lco_feq(int lattice, double rho, const double *u, double *out) {
  lattice_t L;
  if (get_lattice(lattice, &L)) return;
  for (int i = 0; i < L.q; i++) out[i] = feq_i(&L, i, rho, u);
}

void lco_source(int lattice, double tau, const double *u, const double *F, double *out) {
  lattice_t L;
  if (get_lattice(lattice, &L)) return;
  for (int i = 0; i < L.q; i++) out[i] = source_i(&L, i, tau, u, F);
}

/* ---- whole-grid stages --------------------------------------------------- */

/* H (9 per site) and tau (9 per site) from Q. */
static void stage_H_tau(const grid_t *g, const lattice_t *iso, const double *p, const double *q5,
                        double *H9, double *tau9) {
  const size_t N = g->N;
#pragma omp parallel for schedule(static)
  for (size_t s = 0; s < N; s++) {
    double Q[3][3], L[3][3], H[3][3], dQ[3][3][3], tau[3][3];
    full_Q(q5, N, s, Q);
    lap_Q(g, iso, q5, s, L);
    molecular_field(Q, L, p, H);
    grad_Q(g, iso, q5, s, dQ);
    stress(Q, H, dQ, p, tau);
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) {
        if (H9) H9[(a * 3 + b) * N + s] = H[a][b];
        tau9[(a * 3 + b) * N + s] = tau[a][b];
      }
  }
}

/* Body force F_a = d_b tau_ab (central or isotropic differences), then rho
 * and the force-corrected velocity of Eq. (9). */
static void stage_force_moments(const grid_t *g, const lattice_t *L, const lattice_t *iso, const double *tau9,
                                const double *f, double *F3, double *rho1, double *u3) {
  const size_t N = g->N;
#pragma omp parallel for schedule(static)
  for (size_t s = 0; s < N; s++) {
    double F[3];
    for (int a = 0; a < 3; a++) {
      F[a] = 0.0;
      if (iso) {
        for (int i = 1; i < iso->q; i++) {
          const size_t si = displaced(g, s, iso->c[i]);
          for (int b = 0; b < 3; b++) F[a] += iso->w[i] * iso->c[i][b] * tau9[(a * 3 + b) * N + si] / CS2;
        }
        continue;
      }
      for (int b = 0; b < 3; b++) {
        size_t sp = shift(g, s, b, +1), sm = shift(g, s, b, -1);
        F[a] += (tau9[(a * 3 + b) * N + sp] - tau9[(a * 3 + b) * N + sm]) / 2.0;
      }
    }
    if (L->ndim_u == 2) F[2] = 0.0; /* D2Q9 carries no z momentum */
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < L->q; i++) {
      double fi = f[(size_t)i * N + s];
      rho += fi;
      for (int a = 0; a < 3; a++) j[a] += L->c[i][a] * fi;
    }
    rho1[s] = rho;
    for (int a = 0; a < 3; a++) {
      F3[a * N + s] = F[a];
      u3[a * N + s] = (j[a] + F[a] / 2.0) / rho;
    }
  }
}

/* Velocity gradient G[a][b] = d_b u_a at site s (central or isotropic). */
static void velocity_gradient(const grid_t *g, const lattice_t *iso, const double *u3, size_t s, double G[3][3]) {
  const size_t N = g->N;
  if (iso) {
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) G[a][b] = 0.0;
    for (int i = 1; i < iso->q; i++) {
      const size_t si = displaced(g, s, iso->c[i]);
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G[a][b] += iso->w[i] * iso->c[i][b] * u3[a * N + si] / CS2;
    }
    return;
  }
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      size_t sp = shift(g, s, b, +1), sm = shift(g, s, b, -1);
      G[a][b] = (u3[a * N + sp] - u3[a * N + sm]) / 2.0;
    }
}

/* Rate of the five stored components for the tensor field q5, with a given
 * velocity field u3 (3 per site).  Optional full outputs S9, H9. */
static void stage_rate(const grid_t *g, const lattice_t *iso, const double *p, const double *q5, const double *u3,
                       double *R5, double *S9, double *H9) {
  const size_t N = g->N;
#pragma omp parallel for schedule(static)
  for (size_t s = 0; s < N; s++) {
    double Q[3][3], L[3][3], H[3][3], dQ[3][3][3], G[3][3], R[3][3], S[3][3], u[3];
    full_Q(q5, N, s, Q);
    lap_Q(g, iso, q5, s, L);
    molecular_field(Q, L, p, H);
    grad_Q(g, iso, q5, s, dQ);
    velocity_gradient(g, iso, u3, s, G);
    for (int a = 0; a < 3; a++) u[a] = u3[a * N + s];
    be_rate(Q, H, dQ, u, G, p, R, S);
    store5(R, R5, N, s);
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) {
        if (S9) S9[(a * 3 + b) * N + s] = S[a][b];
        if (H9) H9[(a * 3 + b) * N + s] = H[a][b];
      }
  }
}

static int check_args(int lattice, int nx, int ny, int nz, const double *p, lattice_t *L, grid_t *g) {
  if (get_lattice(lattice, L)) return -1;
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  if (lattice == LCO_D2Q9 && nz != 1) return -1;
  if (!(p[5] > 0.5)) return -1;
  g->nx = nx; g->ny = ny; g->nz = nz;
  g->N = (size_t)nx * (size_t)ny * (size_t)nz;
  return 0;
}

/* Intermediate fields of one step at state (f, q5).  Any output may be NULL.
 *   rho[N], u[3N] (force-corrected), F[3N], H[9N], tau[9N], G[9N] (d_b u_a),
 *   R[5N] (rate at Q), Rp[5N] (rate at the predictor), S9[9N] (co-rotational
 *   term at Q). */
int lco_fields(int lattice, int nx, int ny, int nz, const double *p,
               const double *f, const double *q5,
               double *rho_o, double *u_o, double *F_o, double *H_o, double *tau_o,
               double *G_o, double *R_o, double *Rp_o, double *S_o) {
  lattice_t L;
  grid_t g;
  if (check_args(lattice, nx, ny, nz, p, &L, &g)) return -1;
  const size_t N = g.N;
  double *tau9 = malloc(9 * N * sizeof(double));
  double *H9 = malloc(9 * N * sizeof(double));
  double *F3 = malloc(3 * N * sizeof(double));
  double *u3 = malloc(3 * N * sizeof(double));
  double *rho = malloc(N * sizeof(double));
  double *R5 = malloc(5 * N * sizeof(double));
  double *qp = malloc(5 * N * sizeof(double));
  double *Rp5 = malloc(5 * N * sizeof(double));
  if (!tau9 || !H9 || !F3 || !u3 || !rho || !R5 || !qp || !Rp5) return -2;
  const lattice_t *iso = g_stencil ? &L : NULL;
  stage_H_tau(&g, iso, p, q5, H9, tau9);
  stage_force_moments(&g, &L, iso, tau9, f, F3, rho, u3);
  stage_rate(&g, iso, p, q5, u3, R5, S_o, NULL);
  for (size_t k = 0; k < 5 * N; k++) qp[k] = q5[k] + R5[k];
  stage_rate(&g, iso, p, qp, u3, Rp5, NULL, NULL);
  if (rho_o) memcpy(rho_o, rho, N * sizeof(double));
  if (u_o) memcpy(u_o, u3, 3 * N * sizeof(double));
  if (F_o) memcpy(F_o, F3, 3 * N * sizeof(double));
  if (H_o) memcpy(H_o, H9, 9 * N * sizeof(double));
  if (tau_o) memcpy(tau_o, tau9, 9 * N * sizeof(double));
  if (R_o) memcpy(R_o, R5, 5 * N * sizeof(double));
  if (Rp_o) memcpy(Rp_o, Rp5, 5 * N * sizeof(double));
  if (G_o) {
    for (size_t s = 0; s < N; s++) {
      double G[3][3];
      velocity_gradient(&g, iso, u3, s, G);
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G_o[(a * 3 + b) * N + s] = G[a][b];
    }
  }
  free(tau9); free(H9); free(F3); free(u3); free(rho); free(R5); free(qp); free(Rp5);
  return 0;
}

/* Rate R(Q) for a prescribed velocity field u3[3N] (used by consistency
 * checks of the stress against the co-rotational term).  Outputs R5[5N],
 * optional S9[9N] and H9[9N]. */
int lco_rate(int nx, int ny, int nz, const double *p, const double *q5, const double *u3,
             double *R5, double *S9, double *H9) {
  grid_t g;
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.N = (size_t)nx * (size_t)ny * (size_t)nz;
  stage_rate(&g, NULL, p, q5, u3, R5, S9, H9);
  return 0;
}

/* Stress tau[9N] and body force F[3N] of a tensor field (no lattice). */
int lco_stress(int nx, int ny, int nz, const double *p, const double *q5,
               double *tau_o, double *F_o, double *H_o) {
  grid_t g;
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.N = (size_t)nx * (size_t)ny * (size_t)nz;
  const size_t N = g.N;
  double *tau9 = tau_o ? tau_o : malloc(9 * N * sizeof(double));
  stage_H_tau(&g, NULL, p, q5, H_o, tau9);
  if (F_o) {
    for (size_t s = 0; s < N; s++)
      for (int a = 0; a < 3; a++) {
        double F = 0.0;
        for (int b = 0; b < 3; b++) {
          size_t sp = shift(&g, s, b, +1), sm = shift(&g, s, b, -1);
          F += (tau9[(a * 3 + b) * N + sp] - tau9[(a * 3 + b) * N + sm]) / 2.0;
        }
        F_o[a * N + s] = F;
      }
  }
  if (!tau_o) free(tau9);
  return 0;
}

/* ---- multiple-relaxation-time collision (MRT) ------------------------------
 * The paper ran an MRT operator but defers its matrix and rates to another
 * paper (Sec. 1.2.1).  Here the standard orthogonal moment bases: for D2Q9
 * the nine moments of Lallemand and Luo (Phys. Rev. E 61, 6546 (2000)),
 * for D3Q19 the nineteen of d'Humieres et al. (Phil. Trans. R. Soc. A 360,
 * 437 (2002)), each row a polynomial in the lattice velocity c (c2 = |c|^2),
 * listed in the published order:
 *   D2Q9 : rho, e, eps, jx, qx, jy, qy, pxx, pxy
 *   D3Q19: rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww,
 *          pxy, pyz, pxz, mx, my, mz.
 * The collision acts in moment space, m = M f:
 *   m* = m - S (m - M f_eq) + (I - S/2) M G,   f* = M^-1 m*,
 * where S = diag(s_k) and G is the forcing term of Sec. 1.2.1 without its
 * factor (1 - 1/(2 tau)).  With every s_k = 1/tau this is the BGK step
 * above.  The rows of M are orthogonal, so M^-1 = M^T diag(1/|m_k|^2):
 * f*_i = sum_k M_ki (m*_k / |m_k|^2), with the integer entries of M as they
 * are (a numerically computed inverse rounds its entries independently, and
 * its momentum columns then pick up a fixed fraction of the density at every
 * site and step). */
static double basis_row(int lattice, int k, const int c[3]) {
  const double cx = c[0], cy = c[1], cz = c[2];
  const double c2 = cx * cx + cy * cy + cz * cz;
  if (lattice == LCO_D2Q9) {
    switch (k) {
      case 0: return 1.0;
      case 1: return 3.0 * c2 - 4.0;
      case 2: return (9.0 * c2 * c2 - 21.0 * c2 + 8.0) / 2.0;
      case 3: return cx;
      case 4: return (3.0 * c2 - 5.0) * cx;
      case 5: return cy;
      case 6: return (3.0 * c2 - 5.0) * cy;
      case 7: return cx * cx - cy * cy;
      case 8: return cx * cy;
    }
    return 0.0;
  }
  switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return cx;
    case 4: return (5.0 * c2 - 9.0) * cx;
    case 5: return cy;
    case 6: return (5.0 * c2 - 9.0) * cy;
    case 7: return cz;
    case 8: return (5.0 * c2 - 9.0) * cz;
    case 9: return 3.0 * cx * cx - c2;
    case 10: return (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2);
    case 11: return cy * cy - cz * cz;
    case 12: return (3.0 * c2 - 5.0) * (cy * cy - cz * cz);
    case 13: return cx * cy;
    case 14: return cy * cz;
    case 15: return cx * cz;
    case 16: return (cy * cy - cz * cz) * cx;
    case 17: return (cz * cz - cx * cx) * cy;
    case 18: return (cx * cx - cy * cy) * cz;
  }
  return 0.0;
}

/* M[k*q + i] = row k at velocity i.  Returns q, or -1. */
int lco_mrt_basis(int lattice, double *M) {
  lattice_t L;
  if (get_lattice(lattice, &L)) return -1;
  for (int k = 0; k < L.q; k++)
    for (int i = 0; i < L.q; i++) M[k * L.q + i] = basis_row(lattice, k, L.c[i]);
  return L.q;
}

typedef struct {
  double M[19 * 19], norm2[19], s[19]; /* basis, |m_k|^2, rates */
} mrt_t;

/* Post-collision populations at one site with the MRT operator. */
static void collide_mrt(const lattice_t *L, const mrt_t *op, const double *fin, double rho, const double u[3],
                        const double F[3], double *out) {
  const int q = L->q;
  double feq[19], G[19], ms[19];
  for (int i = 0; i < q; i++) {
    feq[i] = feq_i(L, i, rho, u);
    double cu = 0.0, g = 0.0;
    for (int a = 0; a < 3; a++) cu += L->c[i][a] * u[a];
    for (int a = 0; a < 3; a++) g += (L->c[i][a] / CS2 * (1.0 + cu / CS2) - u[a] / CS2) * F[a];
    G[i] = L->w[i] * g;
  }
  for (int k = 0; k < q; k++) {
    double mk = 0.0, mek = 0.0, mgk = 0.0;
    for (int i = 0; i < q; i++) {
      mk += op->M[k * q + i] * fin[i];
      mek += op->M[k * q + i] * feq[i];
      mgk += op->M[k * q + i] * G[i];
    }
    ms[k] = mk - op->s[k] * (mk - mek) + (1.0 - op->s[k] / 2.0) * mgk;
  }
  for (int k = 0; k < q; k++) ms[k] /= op->norm2[k];
  for (int i = 0; i < q; i++) {
    double v = 0.0;
    for (int k = 0; k < q; k++) v += op->M[k * q + i] * ms[k];
    out[i] = v;
  }
}

/* ---- one full time step ---------------------------------------------------
 * Molecular field and stress from Q(n); body force; rho and force-corrected
 * u; Heun predictor-corrector for Q (Sec. 1.2.2 steps 1-5) with u, grad u
 * frozen; BGK collision with forcing; periodic streaming. */
static void one_step(const grid_t *g, const lattice_t *L, const double *p, const mrt_t *op,
                     const double *f, const double *q5, double *f_out, double *q5_out,
                     double *tau9, double *F3, double *rho, double *u3,
                     double *R5, double *qp, double *Rp5) {
  const size_t N = g->N;
  const double tau = p[5];
  const lattice_t *iso = g_stencil ? L : NULL;
  stage_H_tau(g, iso, p, q5, NULL, tau9);
  stage_force_moments(g, L, iso, tau9, f, F3, rho, u3);
  stage_rate(g, iso, p, q5, u3, R5, NULL, NULL);          /* step 1 */
  for (size_t k = 0; k < 5 * N; k++) qp[k] = q5[k] + R5[k]; /* step 2 */
  stage_rate(g, iso, p, qp, u3, Rp5, NULL, NULL);         /* step 3 */
  for (size_t k = 0; k < 5 * N; k++)                 /* steps 4-5 */
    q5_out[k] = q5[k] + (R5[k] + Rp5[k]) / 2.0;
#pragma omp parallel for schedule(static)
  for (size_t s = 0; s < N; s++) {
    double u[3], F[3];
    for (int a = 0; a < 3; a++) {
      u[a] = u3[a * N + s];
      F[a] = F3[a * N + s];
    }
    long x, y, z;
    coords(g, s, &x, &y, &z);
    double fin[19], post[19];
    for (int i = 0; i < L->q; i++) fin[i] = f[(size_t)i * N + s];
    if (op) {
      collide_mrt(L, op, fin, rho[s], u, F, post);
    } else {
      for (int i = 0; i < L->q; i++)
        post[i] = fin[i] - (fin[i] - feq_i(L, i, rho[s], u)) / tau + source_i(L, i, tau, u, F);
    }
    for (int i = 0; i < L->q; i++) {
      size_t d = site(g, x + L->c[i][0], y + L->c[i][1], z + L->c[i][2]);
      f_out[(size_t)i * N + d] = post[i];
    }
  }
}

/* Advance (f, q5) by nsteps in place with the MRT collision when rates
 * (q relaxation rates in the basis order above) is not NULL, else BGK.
 * Returns 0, -1 bad args, -2 no memory. */
int lco_run_coll(int lattice, int nx, int ny, int nz, const double *p, const double *rates, double *f,
                 double *q5, long nsteps) {
  lattice_t L;
  grid_t g;
  if (check_args(lattice, nx, ny, nz, p, &L, &g) || nsteps < 0) return -1;
  mrt_t op, *opp = NULL;
  if (rates) {
    lco_mrt_basis(lattice, op.M);
    for (int k = 0; k < L.q; k++) {
      double n2 = 0.0;
      for (int i = 0; i < L.q; i++) n2 += op.M[k * L.q + i] * op.M[k * L.q + i];
      if (n2 == 0.0) return -1;
      op.norm2[k] = n2;
      op.s[k] = rates[k];
    }
    opp = &op;
  }
  const size_t N = g.N;
  double *f2 = malloc((size_t)L.q * N * sizeof(double));
  double *q2 = malloc(5 * N * sizeof(double));
  double *tau9 = malloc(9 * N * sizeof(double));
  double *F3 = malloc(3 * N * sizeof(double));
  double *rho = malloc(N * sizeof(double));
  double *u3 = malloc(3 * N * sizeof(double));
  double *R5 = malloc(5 * N * sizeof(double));
  double *qp = malloc(5 * N * sizeof(double));
  double *Rp5 = malloc(5 * N * sizeof(double));
  if (!f2 || !q2 || !tau9 || !F3 || !rho || !u3 || !R5 || !qp || !Rp5) return -2;
  for (long n = 0; n < nsteps; n++) {
    one_step(&g, &L, p, opp, f, q5, f2, q2, tau9, F3, rho, u3, R5, qp, Rp5);
    memcpy(f, f2, (size_t)L.q * N * sizeof(double));
    memcpy(q5, q2, 5 * N * sizeof(double));
  }
  free(f2); free(q2); free(tau9); free(F3); free(rho); free(u3); free(R5); free(qp); free(Rp5);
  return 0;
}

/* Advance (f, q5) by nsteps with the BGK collision. */
int lco_run(int lattice, int nx, int ny, int nz, const double *p, double *f, double *q5, long nsteps) {
  return lco_run_coll(lattice, nx, ny, nz, p, NULL, f, q5, nsteps);
}

/* ---- observables ----------------------------------------------------------
 * out[0] mass = sum f; out[1..3] lattice momentum sum c f; out[4] max |u|
 * (force-corrected); out[5] sum of S = sqrt(1.5 Q:Q) over the grid;
 * out[6] sum of S over the half domain c <= coordinate <= c + n/2 along
 * half_axis (end planes weighted 1/2, c = n/2), the trapezoid integral that
 * locates the right-hand interface of a centred slab. */
int lco_observe(int lattice, int nx, int ny, int nz, const double *p,
                const double *f, const double *q5, int half_axis, double *out) {
  lattice_t L;
  grid_t g;
  if (check_args(lattice, nx, ny, nz, p, &L, &g) || half_axis < 0 || half_axis > 2) return -1;
  const size_t N = g.N;
  double *u3 = malloc(3 * N * sizeof(double));
  if (!u3) return -2;
  if (lco_fields(lattice, nx, ny, nz, p, f, q5, NULL, u3, NULL, NULL, NULL, NULL, NULL, NULL, NULL)) {
    free(u3);
    return -1;
  }
  double mass = 0.0, mom[3] = {0, 0, 0}, umax = 0.0, ssum = 0.0, shalf = 0.0;
  int n_ax = half_axis == 0 ? nx : (half_axis == 1 ? ny : nz);
  long c0 = n_ax / 2, c1 = n_ax / 2 + n_ax / 2;
  for (size_t s = 0; s < N; s++) {
    for (int i = 0; i < L.q; i++) {
      double fi = f[(size_t)i * N + s];
      mass += fi;
      for (int a = 0; a < 3; a++) mom[a] += L.c[i][a] * fi;
    }
    double uu = 0.0;
    for (int a = 0; a < 3; a++) uu += u3[a * N + s] * u3[a * N + s];
    if (sqrt(uu) > umax) umax = sqrt(uu);
    double Q[3][3], qq = 0.0;
    full_Q(q5, N, s, Q);
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) qq += Q[a][b] * Q[a][b];
    double S = sqrt(1.5 * qq);
    ssum += S;
    long x, y, z;
    coords(&g, s, &x, &y, &z);
    long k = half_axis == 0 ? x : (half_axis == 1 ? y : z);
    if (k == c0 || k == (c1 % n_ax)) shalf += 0.5 * S;
    else if (k > c0 && k < c1) shalf += S;
  }
  out[0] = mass;
  out[1] = mom[0]; out[2] = mom[1]; out[3] = mom[2];
  out[4] = umax;
  out[5] = ssum;
  out[6] = shalf;
  free(u3);
  return 0;
}
