// lc_staged.h -- the step as four simple sweeps, one site per thread.
//
// Stage kernels keep their intermediates in the caller's scratch buffer:
//   stage_tau  : Q -> stress tau (Eq. 6) at every site;
//   stage_lb   : f, tau -> body force, rho, u (Eq. 9), BGK collision with
//                forcing and push streaming -> f_next; stores u;
//   stage_pred : Q, u -> R(Q) and the predictor Q^P = Q + R (Sec. 1.2.2);
//   stage_corr : Q, Q^P, R, u -> Q_next = Q + (R(Q) + R(Q^P))/2.
// This is the plainest correct mapping of the method onto the GPU; the
// fused and split kernels compute the same per-site arithmetic with fewer
// HBM round trips.  The stage kernels alone also offer the isotropic
// difference stencils (template argument ST, see below).
#pragma once

#include "lc_device.h"

namespace lc {

struct GridDims {
  int nx, ny, nz;
  int64_t N;
};

// Difference stencils.  STENCIL_COMPACT: the central first differences and
// the (2d+1)-point Laplacian of Sec. 1.2.2.  STENCIL_ISO: every derivative
// of the step (grad Q, lap Q, the divergence of the stress, grad u) taken
// from the lattice's own velocities and weights, with c_s^2 = 1/3,
//   d_g V = 3 sum_i w_i c_ig V(x + c_i),   lap V = 6 sum_i w_i [V(x + c_i) - V(x)],
// exact on quadratic fields like the compact ones but with leading errors
// that do not depend on the direction (the remedy for spurious currents
// the closing remarks of Sec. 2.2 point to).  The sums run over pairs of
// opposite velocities: 3 w c_g [V(+c) - V(-c)] and 6 w [(V(+c) - V(x)) +
// (V(-c) - V(x))], the latter differences taken first so that a smooth
// field does not lose its low bits to the sum.
constexpr int STENCIL_COMPACT = 0;
constexpr int STENCIL_ISO = 1;

// Index offset from a site to its neighbour along lattice velocity i.
template <int LAT>
__device__ __forceinline__ int64_t nbr_offset(const Nbr& nb, int i) {
  using L = Lattice<LAT>;
  int64_t d = 0;
  if (L::cx(i) == 1) d += nb.xp;
  if (L::cx(i) == -1) d += nb.xm;
  if (L::cy(i) == 1) d += nb.yp;
  if (L::cy(i) == -1) d += nb.ym;
  if (L::cz(i) == 1) d += nb.zp;
  if (L::cz(i) == -1) d += nb.zm;
  return d;
}

template <int LAT>
__host__ __device__ constexpr int lat_c(int i, int a) {
  return a == 0 ? Lattice<LAT>::cx(i) : (a == 1 ? Lattice<LAT>::cy(i) : Lattice<LAT>::cz(i));
}

// Isotropic gradient and Laplacian of a symmetric tensor field at site s.
template <int LAT, typename S>
__device__ __forceinline__ void stencil_iso(const S* __restrict__ q, int64_t N, int64_t s, const Nbr& nb,
                                            Sym<S>& c, Sym<S> (&d)[3], Sym<S>& L) {
  using Lt = Lattice<LAT>;
  c = load_sym(q, N, s);
  const S cv[5] = {c.xx, c.xy, c.xz, c.yy, c.yz};
  S dv[3][5], lv[5];
#pragma unroll
  for (int k = 0; k < 5; k++) {
    lv[k] = S(0);
#pragma unroll
    for (int g = 0; g < 3; g++) dv[g][k] = S(0);
  }
#pragma unroll
  for (int i = 1; i < Lt::q; i++) {
    if (Lt::opp(i) < i) continue;
    const Sym<S> P = load_sym(q, N, s + nbr_offset<LAT>(nb, i));
    const Sym<S> M = load_sym(q, N, s + nbr_offset<LAT>(nb, Lt::opp(i)));
    const S pv[5] = {P.xx, P.xy, P.xz, P.yy, P.yz}, mv[5] = {M.xx, M.xy, M.xz, M.yy, M.yz};
    const S w3 = S(3.0 * Lt::w(i)), w6 = S(6.0 * Lt::w(i));
#pragma unroll
    for (int k = 0; k < 5; k++) {
      const S diff = pv[k] - mv[k];
#pragma unroll
      for (int g = 0; g < 3; g++)
        if (lat_c<LAT>(i, g) != 0) dv[g][k] += (lat_c<LAT>(i, g) > 0 ? w3 : -w3) * diff;
      lv[k] += w6 * ((pv[k] - cv[k]) + (mv[k] - cv[k]));
    }
  }
#pragma unroll
  for (int g = 0; g < 3; g++) d[g] = Sym<S>{dv[g][0], dv[g][1], dv[g][2], dv[g][3], dv[g][4]};
  L = Sym<S>{lv[0], lv[1], lv[2], lv[3], lv[4]};
}

template <int LAT, typename S, int ST>
__device__ __forceinline__ void stencil_st(const S* __restrict__ q, int64_t N, int64_t s, const Nbr& nb,
                                           Sym<S>& c, Sym<S> (&d)[3], Sym<S>& L) {
  if constexpr (ST == STENCIL_ISO)
    stencil_iso<LAT, S>(q, N, s, nb, c, d, L);
  else
    stencil<S, Lattice<LAT>::dim>(q, N, s, nb, c, d, L);
}

// Number of stress components kept: D2Q9 needs tau_xx, tau_xy, tau_yx,
// tau_yy (the z row of F is not carried); D3Q19 needs all nine.
template <int LAT>
struct TauLayout {
  static constexpr int n = Lattice<LAT>::dim == 2 ? 4 : 9;
  __host__ __device__ static constexpr int idx(int a, int b) {
    return Lattice<LAT>::dim == 2 ? a * 2 + b : a * 3 + b;
  }
};

template <int LAT, typename S, int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(256) stage_tau(const S* __restrict__ Q, S* __restrict__ tau,
                                                 GridDims g, Coef<S> c) {
  constexpr int DIM = Lattice<LAT>::dim;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
  const Nbr nb = neighbours(x, y, z, g.nx, g.ny, g.nz);
  Sym<S> q, L, d[3];
  stencil_st<LAT, S, ST>(Q, g.N, s, nb, q, d, L);
  const Sym<S> H = molecular_field(q, L, c);
  S t[3][3];
  stress(q, H, d, c, t);
  constexpr int D = DIM;
#pragma unroll
  for (int a = 0; a < D; a++)
#pragma unroll
    for (int b = 0; b < D; b++) tau[TauLayout<LAT>::idx(a, b) * g.N + s] = t[a][b];
}

// Body force F_a = sum_b [tau_ab(x+e_b) - tau_ab(x-e_b)]/2 (Sec. 1.2.1),
// or with ST = STENCIL_ISO  F_a = 3 sum_i w_i sum_b c_ib tau_ab(x + c_i).
template <int LAT, typename S, int ST = STENCIL_COMPACT>
__device__ __forceinline__ void body_force(const S* __restrict__ tau, int64_t N, int64_t s, const Nbr& nb,
                                           S (&F)[3]) {
  constexpr int DIM = Lattice<LAT>::dim;
  const int64_t off[3][2] = {{nb.xp, nb.xm}, {nb.yp, nb.ym}, {nb.zp, nb.zm}};
#pragma unroll
  for (int a = 0; a < 3; a++) F[a] = S(0);
  if constexpr (ST == STENCIL_ISO) {
    using Lt = Lattice<LAT>;
#pragma unroll
    for (int i = 1; i < Lt::q; i++) {
      if (Lt::opp(i) < i) continue;
      const int64_t sp = s + nbr_offset<LAT>(nb, i), sm = s + nbr_offset<LAT>(nb, Lt::opp(i));
      const S w3 = S(3.0 * Lt::w(i));
#pragma unroll
      for (int a = 0; a < DIM; a++) {
        S acc = S(0);
#pragma unroll
        for (int b = 0; b < DIM; b++) {
          if (lat_c<LAT>(i, b) == 0) continue;
          const S* t = tau + TauLayout<LAT>::idx(a, b) * N;
          const S dt = t[sp] - t[sm];
          acc += lat_c<LAT>(i, b) > 0 ? dt : -dt;
        }
        F[a] += w3 * acc;
      }
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < DIM; a++) {
    S acc = S(0);
#pragma unroll
    for (int b = 0; b < DIM; b++) {
      const S* t = tau + TauLayout<LAT>::idx(a, b) * N;
      acc += (t[s + off[b][0]] - t[s + off[b][1]]) * S(0.5);
    }
    F[a] = acc;
  }
}

// Density and force-corrected velocity (Eq. 9) from the populations at s.
// With DEV the stored values are f_i - w_i (rho0 = 1); sum_i w_i c_i = 0.
// mass receives the sum of the stored values: rho itself, or in DEV form
// the deviation rho - 1 as summed, which the collision uses for the
// density part of f_eq (forming it again as rho - 1 from the rounded rho
// would lose the deviation's low bits at every site and step).
template <int LAT, typename S, bool DEV>
__device__ __forceinline__ void moments(const S (&f)[Lattice<LAT>::q], const S (&F)[3], S& rho, S (&u)[3],
                                        S& mass) {
  using L = Lattice<LAT>;
  S m = S(0), jx = S(0), jy = S(0), jz = S(0);
#pragma unroll
  for (int i = 0; i < L::q; i++) {
    m += f[i];
    if (L::cx(i) == 1) jx += f[i];
    if (L::cx(i) == -1) jx -= f[i];
    if (L::cy(i) == 1) jy += f[i];
    if (L::cy(i) == -1) jy -= f[i];
    if (L::cz(i) == 1) jz += f[i];
    if (L::cz(i) == -1) jz -= f[i];
  }
  mass = m;
  rho = DEV ? S(1) + m : m;
  const S inv = S(1) / rho;
  u[0] = (jx + S(0.5) * F[0]) * inv;
  u[1] = (jy + S(0.5) * F[1]) * inv;
  u[2] = L::dim == 3 ? (jz + S(0.5) * F[2]) * inv : S(0);
}

template <int LAT, typename S, bool DEV>
__device__ __forceinline__ void moments(const S (&f)[Lattice<LAT>::q], const S (&F)[3], S& rho, S (&u)[3]) {
  S mass;
  moments<LAT, S, DEV>(f, F, rho, u, mass);
}

// BGK collision with the forcing term of Sec. 1.2.1, in place on f.
// Equilibrium Eq. (8) with c_s^2 = 1/3; in DEV form the rest weight w_i is
// removed from both f and f_eq, so only deviations are formed.
// mass: the sum of the stored populations from moments (rho, or rho - 1 in
// DEV form).
template <int LAT, typename S, bool DEV>
__device__ __forceinline__ void collide(S (&f)[Lattice<LAT>::q], S rho, S mass, const S (&u)[3], const S (&F)[3],
                                        const Coef<S>& c) {
  using L = Lattice<LAT>;
  const S uu15 = S(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const S uF3 = S(3) * (u[0] * F[0] + u[1] * F[1] + u[2] * F[2]);
  const S drho = mass;
#pragma unroll
  for (int i = 0; i < L::q; i++) {
    const S w = S(L::w(i));
    const S cu = S(L::cx(i)) * u[0] + S(L::cy(i)) * u[1] + S(L::cz(i)) * u[2];
    const S cF = S(L::cx(i)) * F[0] + S(L::cy(i)) * F[1] + S(L::cz(i)) * F[2];
    // f_eq - (DEV ? w : 0)
    const S feq = DEV ? w * (drho + rho * (S(3) * cu + S(4.5) * cu * cu - uu15))
                      : w * rho * (S(1) + S(3) * cu + S(4.5) * cu * cu - uu15);
    const S src = w * c.src * (S(3) * cF * (S(1) + S(3) * cu) - uF3);
    f[i] = f[i] - c.omega * (f[i] - feq) + src;
  }
}

// The same collision evaluated on pairs of opposite velocities: for c and
// -c the even parts (in c) of f_eq and of the forcing term are shared and
// the odd parts change sign.
template <int LAT, typename S, bool DEV>
__device__ __forceinline__ void collide_pairs(S (&f)[Lattice<LAT>::q], S rho, S mass, const S (&u)[3],
                                              const S (&F)[3], const Coef<S>& c) {
  using L = Lattice<LAT>;
  const S uu15 = S(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const S uF3 = S(3) * (u[0] * F[0] + u[1] * F[1] + u[2] * F[2]);
  const S base = mass;
  const S keep = S(1) - c.omega;
  const S om_rho = c.omega * rho;
  // rest population: c = 0
  {
    const S w = S(L::w(0));
    const S feq = w * (base - rho * uu15);
    f[0] = keep * f[0] + c.omega * feq - w * c.src * uF3;
  }
#pragma unroll
  for (int i = 1; i < L::q; i++) {
    if (L::opp(i) < i) continue;
    const int j = L::opp(i);
    const S w = S(L::w(i));
    const S cu = S(L::cx(i)) * u[0] + S(L::cy(i)) * u[1] + S(L::cz(i)) * u[2];
    const S cF = S(L::cx(i)) * F[0] + S(L::cy(i)) * F[1] + S(L::cz(i)) * F[2];
    const S even = w * (c.omega * base + om_rho * (S(4.5) * cu * cu - uu15) + c.src * (S(9) * cF * cu - uF3));
    const S odd = w * S(3) * (om_rho * cu + c.src * cF);
    const S fi = f[i], fj = f[j];
    f[i] = keep * fi + even + odd;
    f[j] = keep * fj + even - odd;
  }
}

// Multiple-relaxation-time collision with the same forcing.  In moment
// space the step is m* = m - S (m - m_eq) + (I - S/2) M G (G: the forcing
// term without its factor 1 - 1/(2 tau)); with h = f - f_eq + G/2 this is
//   f* = f + G - sum_k s_k P_k h,
// P_k the projector on moment k.  Density, momentum and stress relax at
// omega = 1/tau (h has no density or momentum moment), so
//   f* = [f + G - omega h] - sum_ghosts (s_g - omega) P_k h,
// the bracket being the BGK result.  The ghost projections use the pair
// sums h_i + h_-i for even ghosts and differences for odd ones.
template <int LAT, typename S, bool DEV>
__device__ __forceinline__ void collide_mrt(S (&f)[Lattice<LAT>::q], S rho, S mass, const S (&u)[3],
                                            const S (&F)[3], const Coef<S>& c) {
  using L = Lattice<LAT>;
  using Gh = Ghosts<LAT>;
  const S uu15 = S(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const S uF3 = S(3) * (u[0] * F[0] + u[1] * F[1] + u[2] * F[2]);
  const S base = mass;
  S hs[L::q], hd[L::q];  // per pair representative i: h_i + h_-i, h_i - h_-i; hs[0] = h_0
  {
    const S w = S(L::w(0));
    const S feq = w * (base - rho * uu15);
    const S G = -w * uF3;
    hs[0] = f[0] - feq + S(0.5) * G;
    f[0] = f[0] + G - c.omega * hs[0];
  }
#pragma unroll
  for (int i = 1; i < L::q; i++) {
    if (L::opp(i) < i) continue;
    const int j = L::opp(i);
    const S w = S(L::w(i));
    const S cu = S(L::cx(i)) * u[0] + S(L::cy(i)) * u[1] + S(L::cz(i)) * u[2];
    const S cF = S(L::cx(i)) * F[0] + S(L::cy(i)) * F[1] + S(L::cz(i)) * F[2];
    const S eq_e = w * (base + rho * (S(4.5) * cu * cu - uu15));
    const S eq_o = w * S(3) * rho * cu;
    const S g_e = w * (S(9) * cF * cu - uF3);
    const S g_o = w * S(3) * cF;
    const S hi = f[i] - (eq_e + eq_o) + S(0.5) * (g_e + g_o);
    const S hj = f[j] - (eq_e - eq_o) + S(0.5) * (g_e - g_o);
    f[i] = f[i] + (g_e + g_o) - c.omega * hi;
    f[j] = f[j] + (g_e - g_o) - c.omega * hj;
    hs[i] = hi + hj;
    hd[i] = hi - hj;
  }
  // coefficient of each ghost: (s_g - omega) (m_k . h) / |m_k|^2
  S a[Gh::n];
#pragma unroll
  for (int k = 0; k < Gh::n; k++) {
    S acc = Gh::odd(k) ? S(0) : S(Gh::m(k, 0)) * hs[0];
#pragma unroll
    for (int i = 1; i < L::q; i++) {
      if (L::opp(i) < i || Gh::m(k, i) == 0) continue;
      acc += S(Gh::m(k, i)) * (Gh::odd(k) ? hd[i] : hs[i]);
    }
    a[k] = acc * (c.mrt[Gh::group(k)] * S(1.0 / ghost_norm<LAT>(k)));
  }
  {
    S e = S(0);
#pragma unroll
    for (int k = 0; k < Gh::n; k++)
      if (!Gh::odd(k)) e += a[k] * S(Gh::m(k, 0));
    f[0] -= e;
  }
#pragma unroll
  for (int i = 1; i < L::q; i++) {
    if (L::opp(i) < i) continue;
    S e = S(0), o = S(0);
#pragma unroll
    for (int k = 0; k < Gh::n; k++) {
      if (Gh::m(k, i) == 0) continue;
      if (Gh::odd(k))
        o += a[k] * S(Gh::m(k, i));
      else
        e += a[k] * S(Gh::m(k, i));
    }
    f[i] -= e + o;
    f[L::opp(i)] -= e - o;
  }
}

// Storage convention of the population buffers ("pull" form): the buffer
// of step n holds at site y the post-collision values of step n-1 before
// streaming, so the populations at x are f_i(x) = buf_i(x - c_i).  Kernels
// gather on read and write their post-collision values at their own site,
// which keeps every store aligned and whole.
template <int LAT, typename S>
__device__ __forceinline__ void gather_f(const S* __restrict__ buf, int64_t N, int64_t s, const Nbr& nb,
                                         S (&f)[Lattice<LAT>::q]) {
  using L = Lattice<LAT>;
#pragma unroll
  for (int i = 0; i < L::q; i++) {
    int64_t d = s;
    if (L::cx(i) == 1) d += nb.xm;
    if (L::cx(i) == -1) d += nb.xp;
    if (L::cy(i) == 1) d += nb.ym;
    if (L::cy(i) == -1) d += nb.yp;
    if (L::cz(i) == 1) d += nb.zm;
    if (L::cz(i) == -1) d += nb.zp;
    f[i] = buf[i * N + d];
  }
}

template <int LAT, typename S, bool DEV, bool MRT = false, int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(256) stage_lb(const S* __restrict__ fin, const S* __restrict__ tau,
                                                S* __restrict__ fout, S* __restrict__ uout,
                                                GridDims g, Coef<S> c) {
  using L = Lattice<LAT>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t N = g.N;
  const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
  const Nbr nb = neighbours(x, y, z, g.nx, g.ny, g.nz);
  S F[3];
  body_force<LAT, S, ST>(tau, N, s, nb, F);
  S f[L::q];
  gather_f<LAT, S>(fin, N, s, nb, f);
  S rho, mass, u[3];
  moments<LAT, S, DEV>(f, F, rho, u, mass);
#pragma unroll
  for (int a = 0; a < L::dim; a++) uout[a * N + s] = u[a];
  if constexpr (MRT)
    collide_mrt<LAT, S, DEV>(f, rho, mass, u, F, c);
  else
    collide<LAT, S, DEV>(f, rho, mass, u, F, c);
#pragma unroll
  for (int i = 0; i < L::q; i++) fout[i * N + s] = f[i];
}

// Velocity gradient G[a][b] = d_b u_a (central differences, or with ST =
// STENCIL_ISO 3 sum_i w_i c_ib u_a(x + c_i)).
template <int LAT, typename S, int ST = STENCIL_COMPACT>
__device__ __forceinline__ void velocity_gradient(const S* __restrict__ u, int64_t N, int64_t s, const Nbr& nb,
                                                  S (&G)[3][3], S (&uc)[3]) {
  constexpr int DIM = Lattice<LAT>::dim;
  if constexpr (ST == STENCIL_ISO) {
    using Lt = Lattice<LAT>;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      uc[a] = a < DIM ? u[a * N + s] : S(0);
#pragma unroll
      for (int b = 0; b < 3; b++) G[a][b] = S(0);
    }
#pragma unroll
    for (int i = 1; i < Lt::q; i++) {
      if (Lt::opp(i) < i) continue;
      const int64_t sp = s + nbr_offset<LAT>(nb, i), sm = s + nbr_offset<LAT>(nb, Lt::opp(i));
      const S w3 = S(3.0 * Lt::w(i));
#pragma unroll
      for (int a = 0; a < DIM; a++) {
        const S du = w3 * (u[a * N + sp] - u[a * N + sm]);
#pragma unroll
        for (int b = 0; b < DIM; b++)
          if (lat_c<LAT>(i, b) != 0) G[a][b] += lat_c<LAT>(i, b) > 0 ? du : -du;
      }
    }
    return;
  }
  const int64_t off[3][2] = {{nb.xp, nb.xm}, {nb.yp, nb.ym}, {nb.zp, nb.zm}};
#pragma unroll
  for (int a = 0; a < 3; a++) {
    uc[a] = a < DIM ? u[a * N + s] : S(0);
#pragma unroll
    for (int b = 0; b < 3; b++)
      G[a][b] = (a < DIM && b < DIM) ? (u[a * N + s + off[b][0]] - u[a * N + s + off[b][1]]) * S(0.5) : S(0);
  }
}

template <int LAT, typename S, int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(256) stage_pred(const S* __restrict__ Q, const S* __restrict__ u,
                                                  S* __restrict__ qp, S* __restrict__ rq, GridDims g,
                                                  Coef<S> c) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
  const Nbr nb = neighbours(x, y, z, g.nx, g.ny, g.nz);
  Sym<S> q, L, d[3];
  stencil_st<LAT, S, ST>(Q, g.N, s, nb, q, d, L);
  const Sym<S> H = molecular_field(q, L, c);
  S G[3][3], uc[3];
  velocity_gradient<LAT, S, ST>(u, g.N, s, nb, G, uc);
  const Sym<S> R = be_rate(q, H, d, uc, G, c);
  store_sym(rq, g.N, s, R);
  store_sym(qp, g.N, s, Sym<S>{q.xx + R.xx, q.xy + R.xy, q.xz + R.xz, q.yy + R.yy, q.yz + R.yz});
}

template <int LAT, typename S, int ST = STENCIL_COMPACT>
__global__ void __launch_bounds__(256) stage_corr(const S* __restrict__ Q, const S* __restrict__ qp,
                                                  const S* __restrict__ rq, const S* __restrict__ u,
                                                  S* __restrict__ Qout, GridDims g, Coef<S> c) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t s = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
  const Nbr nb = neighbours(x, y, z, g.nx, g.ny, g.nz);
  Sym<S> p, L, d[3];
  stencil_st<LAT, S, ST>(qp, g.N, s, nb, p, d, L);
  const Sym<S> H = molecular_field(p, L, c);
  S G[3][3], uc[3];
  velocity_gradient<LAT, S, ST>(u, g.N, s, nb, G, uc);
  const Sym<S> Rp = be_rate(p, H, d, uc, G, c);
  const Sym<S> q = load_sym(Q, g.N, s);
  const Sym<S> R = load_sym(rq, g.N, s);
  store_sym(Qout, g.N, s,
            Sym<S>{q.xx + S(0.5) * (R.xx + Rp.xx), q.xy + S(0.5) * (R.xy + Rp.xy),
                   q.xz + S(0.5) * (R.xz + Rp.xz), q.yy + S(0.5) * (R.yy + Rp.yy),
                   q.yz + S(0.5) * (R.yz + Rp.yz)});
}

}  // namespace lc
