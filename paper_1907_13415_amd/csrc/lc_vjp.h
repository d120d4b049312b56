// lc_vjp.h -- one reverse-mode step of the hybrid scheme (D2Q9, double).
//
// Given the state (f, Q) at step n (logical populations, before collision)
// and the adjoint (adj_f, adj_Q) of the state at step n+1, the kernels
// below overwrite the adjoint with that of step n and accumulate the
// derivatives with respect to gamma, K and Gamma.  The forward quantities
// of the step (stress, density, velocity, body force, predictor) are
// recomputed first; the reverse sweep then runs the chain backwards:
//   streaming and collision -> corrector rate at Q^P (and its H, Laplacian
//   and gradient stencils) -> predictor rate at Q -> velocity gradient and
//   force-corrected velocity -> body force and stress -> molecular field.
// Stencil adjoints are applied as gathers: the compact Laplacian is
// self-adjoint and the central difference D has adjoint -D on a periodic
// grid.  The three kernels of a reverse step run two threads per site: the
// block is REV_TX x REV_TY sites by two halves (threadIdx.z), each half
// takes an independent part of the site's work, and the halves meet in LDS
// (a grid of 65 536 sites would otherwise give one wave per SIMD).  Each
// value is formed by the same operations in the same order as with one
// thread per site, so the split does not change any result.
#pragma once

#include "lc_adjoint.h"
#include "lc_aux.h"

namespace lc {

// Scratch fields of the reverse step (double, N values per component).
struct VjpFields {
  double *tau, *rho, *u, *F, *qp, *r;                 // forward recompute
  double *fbar, *qpb, *lpb, *dqpb, *ub, *gb, *rhob;  // reverse
  double *fb, *qb, *hb, *dqb, *lb;
  double *part;  // [3 kernels][nblocks][3] parameter partials
  int64_t nblocks;
};
constexpr int VJP_COMPS = 4 + 1 + 2 + 2 + 5 + 5 + 9 + 5 + 5 + 10 + 2 + 4 + 1 + 2 + 5 + 5 + 10 + 5;

// sites per block of the reverse kernels (the block has two halves)
constexpr int REV_TX = 64, REV_TY = 4, REV_SITES = REV_TX * REV_TY;

__device__ __forceinline__ void block_reduce3(double (&v)[3], double* __restrict__ dst) {
  __shared__ double part[16][3];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int lane = tid & 63, wid = tid >> 6;
  const int nw = (blockDim.x * blockDim.y * blockDim.z + 63) >> 6;
#pragma unroll
  for (int k = 0; k < 3; k++) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 3; k++) part[wid][k] = v[k];
  }
  __syncthreads();
  if (tid < 3) {
    double acc = part[0][tid];
    for (int w = 1; w < nw; w++) acc += part[w][tid];
    dst[tid] += acc;  // accumulate over the reverse steps of one call
  }
}

// zero the per-block parameter partials before a reverse call
__global__ void __launch_bounds__(256) vjp_zero(double* __restrict__ part, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    part[i] = 0.0;
}

// Laplacian and minus-divergence gathers of adjoint fields at site s.
__device__ __forceinline__ Sym<double> lap2(const double* __restrict__ A, int64_t N, int64_t s, const Nbr& nb) {
  auto one = [&](int c) {
    const double* a = A + c * N;
    return (a[s + nb.xp] + a[s + nb.xm]) + (a[s + nb.yp] + a[s + nb.ym]) - 4.0 * a[s];
  };
  return Sym<double>{one(0), one(1), one(2), one(3), one(4)};
}

// -sum_g D_g(W_g) for W laid out [g][5][N], g = x, y
__device__ __forceinline__ Sym<double> negdiv2(const double* __restrict__ W, int64_t N, int64_t s, const Nbr& nb) {
  auto one = [&](int c) {
    const double* wx = W + (0 * 5 + c) * N;
    const double* wy = W + (1 * 5 + c) * N;
    return -0.5 * ((wx[s + nb.xp] - wx[s + nb.xm]) + (wy[s + nb.yp] - wy[s + nb.ym]));
  };
  return Sym<double>{one(0), one(1), one(2), one(3), one(4)};
}

__device__ __forceinline__ void put5(double* __restrict__ A, int64_t N, int64_t s, const Sym<double>& v) {
  A[s] = v.xx;
  A[N + s] = v.xy;
  A[2 * N + s] = v.xz;
  A[3 * N + s] = v.yy;
  A[4 * N + s] = v.yz;
}

__device__ __forceinline__ void velgrad2(const double* __restrict__ u, int64_t N, int64_t s, const Nbr& nb,
                                         double (&G)[3][3], double (&uc)[3]) {
#pragma unroll
  for (int a = 0; a < 3; a++) {
    uc[a] = a < 2 ? u[a * N + s] : 0.0;
    for (int b = 0; b < 3; b++) G[a][b] = 0.0;
  }
#pragma unroll
  for (int a = 0; a < 2; a++) {
    G[a][0] = 0.5 * (u[a * N + s + nb.xp] - u[a * N + s + nb.xm]);
    G[a][1] = 0.5 * (u[a * N + s + nb.yp] - u[a * N + s + nb.ym]);
  }
}

#define LC_SITE_2D                                                       \
  const int x = blockIdx.x * blockDim.x + threadIdx.x;                   \
  const int y = blockIdx.y * blockDim.y + threadIdx.y;                   \
  const bool in = x < g.nx && y < g.ny;                                  \
  const int64_t N = g.N;                                                 \
  const int64_t s = in ? x + (int64_t)g.nx * y : 0;                      \
  const Nbr nb = neighbours(in ? x : 0, in ? y : 0, 0, g.nx, g.ny, 1);   \
  const int64_t blk = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;

// density, force-corrected velocity and body force from f and tau; f is
// either logical (pull == 0) or a population buffer in pull form
__global__ void __launch_bounds__(256) vjp_fwd_moments(const double* __restrict__ f, int pull,
                                                       const double* __restrict__ tau, VjpFields v, GridDims g) {
  LC_SITE_2D
  (void)blk;
  if (!in) return;
  double F[3];
  body_force<0, double>(tau, N, s, nb, F);
  double ff[9];
  if (pull) {
    gather_f<0, double>(f, N, s, nb, ff);
  } else {
#pragma unroll
    for (int i = 0; i < 9; i++) ff[i] = f[i * N + s];
  }
  double rho, u[3];
  moments<0, double, false>(ff, F, rho, u);
  v.rho[s] = rho;
  v.u[s] = u[0];
  v.u[N + s] = u[1];
  v.F[s] = F[0];
  v.F[N + s] = F[1];
}

// collision and corrector-rate adjoints.  With fold set, the order-tensor
// adjoint is first assembled from the previous reverse step's qb, lb, dqb
// (the Laplacian and gradient gathers of vjp_r5) and stored to adj_q; the
// gathered fields are only read here, and adj_q only at the own site.
// Half 0 takes the collision, half 1 the corrector; the velocity adjoint is
// the sum of the two (collision first).
__global__ void __launch_bounds__(2 * REV_SITES) vjp_r1(const double* __restrict__ adj_f, double* __restrict__ adj_q,
                                                        int fold, VjpFields v, GridDims g, Coef<double> c) {
  using L = Lattice<0>;
  LC_SITE_2D
  const int half = threadIdx.z;
  const int slot = threadIdx.x + blockDim.x * threadIdx.y;
  __shared__ double s_ub[2][REV_SITES];
  double d[3] = {0.0, 0.0, 0.0};
  double ub[3] = {0.0, 0.0, 0.0};
  if (in && half == 0) {
    double fbs[9];
#pragma unroll
    for (int i = 0; i < 9; i++) {
      int64_t t = s;
      if (L::cx(i) == 1) t += nb.xp;
      if (L::cx(i) == -1) t += nb.xm;
      if (L::cy(i) == 1) t += nb.yp;
      if (L::cy(i) == -1) t += nb.ym;
      fbs[i] = adj_f[i * N + t];  // f'_i(x + c_i) = f*_i(x)
    }
    const double rho = v.rho[s];
    const double u3[3] = {v.u[s], v.u[N + s], 0.0};
    const double F3[3] = {v.F[s], v.F[N + s], 0.0};
    double fb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, rhob = 0.0, ubc[3] = {0, 0, 0}, Fb[3] = {0, 0, 0};
    collide_vjp<0, double>(fbs, rho, u3, F3, c, fb, rhob, ubc, Fb);
#pragma unroll
    for (int i = 0; i < 9; i++) v.fbar[i * N + s] = fb[i];
    v.rhob[s] = rhob;
    v.fb[s] = Fb[0];
    v.fb[N + s] = Fb[1];
    s_ub[0][slot] = ubc[0];
    s_ub[1][slot] = ubc[1];
  }
  if (in && half == 1) {
    Sym<double> aq;
    if (fold) {
      aq = load_sym(v.qb, N, s);
      add_to(aq, lap2(v.lb, N, s, nb));
      add_to(aq, negdiv2(v.dqb, N, s, nb));
      put5(adj_q, N, s, aq);
    } else {
      aq = load_sym(adj_q, N, s);
    }
    // corrector: Q' = Q + (R + R^P)/2
    const Sym<double> Rpb{0.5 * aq.xx, 0.5 * aq.xy, 0.5 * aq.xz, 0.5 * aq.yy, 0.5 * aq.yz};
    Sym<double> P, dP[3], LP;
    stencil<double, 2>(v.qp, N, s, nb, P, dP, LP);
    const Sym<double> HP = molecular_field(P, LP, c);
    double G[3][3], uc[3];
    velgrad2(v.u, N, s, nb, G, uc);
    Sym<double> Pb = sym_zero<double>(), HPb = sym_zero<double>(), LPb;
    Sym<double> dPb[3] = {sym_zero<double>(), sym_zero<double>(), sym_zero<double>()};
    double Gb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    be_rate_vjp(P, HP, dP, uc, G, Rpb, c, Pb, HPb, dPb, ub, Gb, d);
    molecular_field_vjp(P, LP, HPb, c, Pb, LPb, d);
    put5(v.qpb, N, s, Pb);
    put5(v.lpb, N, s, LPb);
    put5(v.dqpb, N, s, dPb[0]);
    put5(v.dqpb + 5 * N, N, s, dPb[1]);
    v.gb[s] = Gb[0][0];
    v.gb[N + s] = Gb[0][1];
    v.gb[2 * N + s] = Gb[1][0];
    v.gb[3 * N + s] = Gb[1][1];
  }
  __syncthreads();
  if (in && half == 1) {
    // ub holds the corrector's part alone (it started from zero and was
    // decremented once per component), so adding it to the collision's part
    // rounds as decrementing that part would
    v.ub[s] = s_ub[0][slot] + ub[0];
    v.ub[N + s] = s_ub[1][slot] + ub[1];
  }
  block_reduce3(d, v.part + (0 * v.nblocks + blk) * 3);
}

// predictor-rate adjoint at Q.  Half 0 gathers the predictor's adjoint and
// forms the rate adjoint; half 1 evaluates the stencil, H and the velocity
// gradient at Q, then takes the rate adjoint from LDS.
__global__ void __launch_bounds__(2 * REV_SITES) vjp_r2(const double* __restrict__ Q, const double* __restrict__ adj_q,
                                                        VjpFields v, GridDims g, Coef<double> c) {
  LC_SITE_2D
  const int half = threadIdx.z;
  const int slot = threadIdx.x + blockDim.x * threadIdx.y;
  __shared__ double s_rb[5][REV_SITES], s_qb[5][REV_SITES];
  double d[3] = {0.0, 0.0, 0.0};
  Sym<double> q, dq[3], Lq, H;
  double G[3][3], uc[3];
  if (in && half == 0) {
    Sym<double> qpb = load_sym(v.qpb, N, s);
    add_to(qpb, lap2(v.lpb, N, s, nb));
    add_to(qpb, negdiv2(v.dqpb, N, s, nb));
    const Sym<double> aq = load_sym(adj_q, N, s);
    const double rb[5] = {0.5 * aq.xx + qpb.xx, 0.5 * aq.xy + qpb.xy, 0.5 * aq.xz + qpb.xz, 0.5 * aq.yy + qpb.yy,
                          0.5 * aq.yz + qpb.yz};
    const double qb[5] = {aq.xx + qpb.xx, aq.xy + qpb.xy, aq.xz + qpb.xz, aq.yy + qpb.yy, aq.yz + qpb.yz};
#pragma unroll
    for (int k = 0; k < 5; k++) {
      s_rb[k][slot] = rb[k];
      s_qb[k][slot] = qb[k];
    }
  }
  if (in && half == 1) {
    stencil<double, 2>(Q, N, s, nb, q, dq, Lq);
    H = molecular_field(q, Lq, c);
    velgrad2(v.u, N, s, nb, G, uc);
  }
  __syncthreads();
  if (in && half == 1) {
    const Sym<double> Rb{s_rb[0][slot], s_rb[1][slot], s_rb[2][slot], s_rb[3][slot], s_rb[4][slot]};
    Sym<double> qb{s_qb[0][slot], s_qb[1][slot], s_qb[2][slot], s_qb[3][slot], s_qb[4][slot]};
    Sym<double> Hb = sym_zero<double>();
    Sym<double> dqb[3] = {sym_zero<double>(), sym_zero<double>(), sym_zero<double>()};
    double ub[3] = {v.ub[s], v.ub[N + s], 0.0};
    double Gb[3][3] = {{v.gb[s], v.gb[N + s], 0.0}, {v.gb[2 * N + s], v.gb[3 * N + s], 0.0}, {0, 0, 0}};
    be_rate_vjp(q, H, dq, uc, G, Rb, c, qb, Hb, dqb, ub, Gb, d);
    put5(v.qb, N, s, qb);
    put5(v.hb, N, s, Hb);
    put5(v.dqb, N, s, dqb[0]);
    put5(v.dqb + 5 * N, N, s, dqb[1]);
    v.ub[s] = ub[0];
    v.ub[N + s] = ub[1];
    v.gb[s] = Gb[0][0];
    v.gb[N + s] = Gb[0][1];
    v.gb[2 * N + s] = Gb[1][0];
    v.gb[3 * N + s] = Gb[1][1];
  }
  block_reduce3(d, v.part + (1 * v.nblocks + blk) * 3);
}

// Adjoint of the force-corrected momentum at site t (neighbour offsets nt):
// the velocity adjoint with the velocity-gradient gather applied, over rho.
__device__ __forceinline__ void momentum_adj(const VjpFields& v, int64_t N, int64_t t, const Nbr& nt,
                                             double (&ub)[2], double (&jb)[2]) {
#pragma unroll
  for (int a = 0; a < 2; a++) {
    const double* gx = v.gb + (a * 2 + 0) * N;  // G_{a x}
    const double* gy = v.gb + (a * 2 + 1) * N;  // G_{a y}
    ub[a] = v.ub[a * N + t] - 0.5 * ((gx[t + nt.xp] - gx[t + nt.xm]) + (gy[t + nt.yp] - gy[t + nt.ym]));
  }
  const double rho = v.rho[t];
  jb[0] = ub[0] / rho;
  jb[1] = ub[1] / rho;
}

// adjoint of the body force at site t (the force enters u with weight 1/2)
__device__ __forceinline__ void force_adj(const VjpFields& v, const GridDims& g, int x, int y, double (&fb2)[2]) {
  const int64_t t = x + (int64_t)g.nx * y;
  const Nbr nt = neighbours(x, y, 0, g.nx, g.ny, 1);
  double ub[2], jb[2];
  momentum_adj(v, g.N, t, nt, ub, jb);
  fb2[0] = v.fb[t] + 0.5 * jb[0];
  fb2[1] = v.fb[g.N + t] + 0.5 * jb[1];
}

// Velocity-gradient and moment adjoints (writes the population adjoint),
// then body-force, stress and molecular-field adjoints at Q.  The force
// adjoint of the four neighbours is recomputed here rather than stored.
// Half 0 takes the population adjoint and the stress adjoint (from the four
// neighbours' force adjoints); half 1 evaluates the stencil and H at Q and
// then the stress and molecular-field adjoints.
__global__ void __launch_bounds__(2 * REV_SITES) vjp_r34(double* __restrict__ adj_f, const double* __restrict__ Q,
                                                         VjpFields v, GridDims g, Coef<double> c) {
  using L = Lattice<0>;
  LC_SITE_2D
  const int half = threadIdx.z;
  const int slot = threadIdx.x + blockDim.x * threadIdx.y;
  __shared__ double s_tb[4][REV_SITES];
  double d[3] = {0.0, 0.0, 0.0};
  Sym<double> q, dq[3], Lq, H;
  if (in && half == 0) {
    {
      double ub[2], jb[2];
      momentum_adj(v, N, s, nb, ub, jb);
      const double rhob = v.rhob[s] - (ub[0] * v.u[s] + ub[1] * v.u[N + s]) / v.rho[s];
#pragma unroll
      for (int i = 0; i < 9; i++) adj_f[i * N + s] = v.fbar[i * N + s] + rhob + L::cx(i) * jb[0] + L::cy(i) * jb[1];
    }
    const int xp = x + 1 == g.nx ? 0 : x + 1, xm = x == 0 ? g.nx - 1 : x - 1;
    const int yp = y + 1 == g.ny ? 0 : y + 1, ym = y == 0 ? g.ny - 1 : y - 1;
    double fxp[2], fxm[2], fyp[2], fym[2];
    force_adj(v, g, xp, y, fxp);
    force_adj(v, g, xm, y, fxm);
    force_adj(v, g, x, yp, fyp);
    force_adj(v, g, x, ym, fym);
#pragma unroll
    for (int a = 0; a < 2; a++) {
      s_tb[2 * a + 0][slot] = -0.5 * (fxp[a] - fxm[a]);
      s_tb[2 * a + 1][slot] = -0.5 * (fyp[a] - fym[a]);
    }
  }
  if (in && half == 1) {
    stencil<double, 2>(Q, N, s, nb, q, dq, Lq);
    H = molecular_field(q, Lq, c);
  }
  __syncthreads();
  if (in && half == 1) {
    double tb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int a = 0; a < 2; a++) {
      tb[a][0] = s_tb[2 * a + 0][slot];
      tb[a][1] = s_tb[2 * a + 1][slot];
    }
    Sym<double> qb = load_sym(v.qb, N, s);
    Sym<double> Hb = load_sym(v.hb, N, s);
    Sym<double> dqb[3] = {load_sym(v.dqb, N, s), load_sym(v.dqb + 5 * N, N, s), sym_zero<double>()};
    stress_vjp(q, H, dq, tb, c, qb, Hb, dqb, d);
    Sym<double> Lb;
    molecular_field_vjp(q, Lq, Hb, c, qb, Lb, d);
    put5(v.qb, N, s, qb);
    put5(v.lb, N, s, Lb);
    put5(v.dqb, N, s, dqb[0]);
    put5(v.dqb + 5 * N, N, s, dqb[1]);
  }
  block_reduce3(d, v.part + (2 * v.nblocks + blk) * 3);
}

// Laplacian and gradient gathers into the order-tensor adjoint
__global__ void __launch_bounds__(256) vjp_r5(double* __restrict__ adj_q, VjpFields v, GridDims g) {
  LC_SITE_2D
  (void)blk;
  if (!in) return;
  Sym<double> qb = load_sym(v.qb, N, s);
  add_to(qb, lap2(v.lb, N, s, nb));
  add_to(qb, negdiv2(v.dqb, N, s, nb));
  put5(adj_q, N, s, qb);
}

// parameter partials of the three kernels, added to dparams: each thread
// sums a fixed strided subset, then a fixed-order block reduction
// (deterministic for a fixed launch shape).
__global__ void __launch_bounds__(256) vjp_params(const double* __restrict__ part, int64_t nblocks,
                                                  double* __restrict__ dparams) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < 3 * nblocks; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 3; k++) v[k] += part[b * 3 + k];
  }
  __shared__ double tot[3];
  if (threadIdx.x < 3) tot[threadIdx.x] = 0.0;
  __syncthreads();
  block_reduce3(v, tot);
  __syncthreads();
  if (threadIdx.x < 3) dparams[threadIdx.x] += tot[threadIdx.x];
}

}  // namespace lc
