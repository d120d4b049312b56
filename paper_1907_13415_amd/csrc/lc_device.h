// lc_device.h -- per-site device arithmetic of the hybrid LB / FD step.
//
// Everything here is inlined into the kernels.  Symmetric traceless tensors
// are carried as five values (xx, xy, xz, yy, yz), zz = -xx - yy, and the
// tensor algebra of Eqs. (2), (4) and (6) is written out using that symmetry
// rather than as 3x3 loops.  T is the arithmetic type (double for LC_FP64,
// float for LC_FP32_DEV).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Per-site helpers are usable from host code too (the adjoint unit checks
// run them on the CPU).
#define LC_HD __host__ __device__ __forceinline__

namespace lc {

// ---------------------------------------------------------------------------
// Velocity sets.  c_s^2 = 1/3 (Sec. 1.2.1).  The order is part of the ABI.
template <int LAT>
struct Lattice;

template <>
struct Lattice<0> {  // D2Q9
  static constexpr int q = 9;
  static constexpr int dim = 2;
  __host__ __device__ static constexpr int cx(int i) {
    return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int i) {
    return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  // index of the velocity -c_i
  __host__ __device__ static constexpr int opp(int i) {
    return i == 0 ? 0 : (i < 5 ? (i <= 2 ? i + 2 : i - 2) : (i <= 6 ? i + 2 : i - 2));
  }
};

template <>
struct Lattice<1> {  // D3Q19
  static constexpr int q = 19;
  static constexpr int dim = 3;
  // rest; +-x, +-y, +-z; xy edges; xz edges; yz edges
  __host__ __device__ static constexpr int cx(int i) {
    return i == 1 || i == 7 || i == 9 || i == 11 || i == 13
               ? 1
               : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14 ? -1 : 0);
  }
  __host__ __device__ static constexpr int cy(int i) {
    return i == 3 || i == 7 || i == 10 || i == 15 || i == 17
               ? 1
               : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18 ? -1 : 0);
  }
  __host__ __device__ static constexpr int cz(int i) {
    return i == 5 || i == 11 || i == 14 || i == 15 || i == 18
               ? 1
               : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17 ? -1 : 0);
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  // index of the velocity -c_i (pairs are adjacent: odd i pairs with i + 1)
  __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
};

// ---------------------------------------------------------------------------
// Non-hydrodynamic ("ghost") moments of the standard orthogonal MRT bases:
// Lallemand and Luo (2000) for D2Q9, d'Humieres et al. (2002) for D3Q19.
// Each is a polynomial in the lattice velocity (c2 = |c|^2); the remaining
// moments of those bases are density, momentum and the traceless stress,
// which the collision treats as in BGK (stress relaxed at 1/tau).  A ghost
// belongs to a rate group; even ghosts do not change sign under c -> -c,
// odd ones do.
template <int LAT>
struct Ghosts;

template <>
struct Ghosts<0> {  // e, eps, qx, qy; groups e, eps, q
  static constexpr int n = 4;
  static constexpr int ngroups = 3;
  __host__ __device__ static constexpr int group(int k) { return k < 2 ? k : 2; }
  __host__ __device__ static constexpr bool odd(int k) { return k >= 2; }
  __host__ __device__ static constexpr int m(int k, int i) {
    using L = Lattice<0>;
    const int cx = L::cx(i), cy = L::cy(i), c2 = cx * cx + cy * cy;
    return k == 0 ? 3 * c2 - 4 : (k == 1 ? (9 * c2 * c2 - 21 * c2 + 8) / 2 : (3 * c2 - 5) * (k == 2 ? cx : cy));
  }
};

template <>
struct Ghosts<1> {  // e, eps, qx, qy, qz, 3pixx, piww, mx, my, mz; groups e, eps, q, pi, m
  static constexpr int n = 10;
  static constexpr int ngroups = 5;
  __host__ __device__ static constexpr int group(int k) {
    return k < 2 ? k : (k < 5 ? 2 : (k < 7 ? 3 : 4));
  }
  __host__ __device__ static constexpr bool odd(int k) { return (k >= 2 && k < 5) || k >= 7; }
  __host__ __device__ static constexpr int m(int k, int i) {
    using L = Lattice<1>;
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    const int xx = cx * cx, yy = cy * cy, zz = cz * cz, c2 = xx + yy + zz;
    switch (k) {
      case 0: return 19 * c2 - 30;
      case 1: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
      case 2: return (5 * c2 - 9) * cx;
      case 3: return (5 * c2 - 9) * cy;
      case 4: return (5 * c2 - 9) * cz;
      case 5: return (3 * c2 - 5) * (3 * xx - c2);
      case 6: return (3 * c2 - 5) * (yy - zz);
      case 7: return (yy - zz) * cx;
      case 8: return (zz - xx) * cy;
      default: return (xx - yy) * cz;
    }
  }
};

// Squared norm of ghost k over the velocity set.
template <int LAT>
__host__ __device__ constexpr int ghost_norm(int k) {
  int s = 0;
  for (int i = 0; i < Lattice<LAT>::q; i++) s += Ghosts<LAT>::m(k, i) * Ghosts<LAT>::m(k, i);
  return s;
}

// ---------------------------------------------------------------------------
// Per-launch constants derived from lc_params (in the arithmetic type).
template <typename T>
struct Coef {
  T lin;     // -A0 (1 - gamma/3): coefficient of Q in H
  T quad;    // A0 gamma: coefficient of Q.Q (and -1/3 of its trace) in H
  T K;       // elastic constant
  T Gam;     // rotational diffusion
  T xi;      // flow alignment
  T xi_p;    // (xi + 1)/2
  T xi_m;    // (xi - 1)/2
  T omega;   // 1/tau
  T src;     // 1 - 1/(2 tau)
  T A0;      // bulk coefficient (the adjoint needs d/dgamma of lin and quad)
  // MRT: rate of each ghost group minus 1/tau (unused by the BGK kernels)
  T mrt[5];
  // lin and quad unrounded, for the bulk part of the molecular field of the
  // float form with stochastic rounding (evaluated in double there)
  double lin_d, quad_d;
};

template <typename T>
struct Sym {
  T xx, xy, xz, yy, yz;
  LC_HD T zz() const { return -xx - yy; }
};

template <typename T>
LC_HD Sym<T> sym_zero() {
  return Sym<T>{T(0), T(0), T(0), T(0), T(0)};
}

// Full contraction A:B of two symmetric traceless tensors.
template <typename T>
LC_HD T ddot(const Sym<T>& a, const Sym<T>& b) {
  return a.xx * b.xx + a.yy * b.yy + (a.xx + a.yy) * (b.xx + b.yy) +
         T(2) * (a.xy * b.xy + a.xz * b.xz + a.yz * b.yz);
}

// Molecular field, Eq. (4), from Q and its Laplacian L, evaluated in type
// E with coefficients lin, quad, K:
//   H = lin Q + quad (Q.Q - Tr(Q^2) I/3) - quad Tr(Q^2) Q + K L.
template <typename E, typename T>
LC_HD Sym<T> molecular_field_in(const Sym<T>& Qt, const Sym<T>& Lt, E lin, E quad, E K) {
  const Sym<E> Q{E(Qt.xx), E(Qt.xy), E(Qt.xz), E(Qt.yy), E(Qt.yz)};
  const E zz = Q.zz();
  const E sxx = Q.xx * Q.xx + Q.xy * Q.xy + Q.xz * Q.xz;
  const E syy = Q.xy * Q.xy + Q.yy * Q.yy + Q.yz * Q.yz;
  const E szz = Q.xz * Q.xz + Q.yz * Q.yz + zz * zz;
  const E sxy = Q.xx * Q.xy + Q.xy * Q.yy + Q.xz * Q.yz;
  const E sxz = Q.xx * Q.xz + Q.xy * Q.yz + Q.xz * zz;
  const E syz = Q.xy * Q.xz + Q.yy * Q.yz + Q.yz * zz;
  const E tr2 = sxx + syy + szz;
  const E a = lin - quad * tr2;
  const E third = quad * tr2 * E(1.0 / 3.0);
  // grouped so that each component is one chain of fused multiply-adds
  Sym<T> H;
  H.xx = T(a * Q.xx + (quad * sxx + (K * E(Lt.xx) - third)));
  H.yy = T(a * Q.yy + (quad * syy + (K * E(Lt.yy) - third)));
  H.xy = T(a * Q.xy + (quad * sxy + K * E(Lt.xy)));
  H.xz = T(a * Q.xz + (quad * sxz + K * E(Lt.xz)));
  H.yz = T(a * Q.yz + (quad * syz + K * E(Lt.yz)));
  return H;
}

template <typename T>
LC_HD Sym<T> molecular_field(const Sym<T>& Q, const Sym<T>& L, const Coef<T>& c) {
  return molecular_field_in<T, T>(Q, L, c.lin, c.quad, c.K);
}

// The molecular field of the float form with stochastic rounding: the bulk
// terms nearly cancel near the nematic minimum, and their float rounding,
// the same at a site from one step to the next while the state there is
// unchanged, acts as a small systematic force; so does the rounding of the
// bulk coefficients, which shifts the coexistence temperature.  The bulk
// part is summed in double from the float Q with the unrounded
// coefficients and rounded once; K L is then added in float.
template <typename T>
LC_HD Sym<T> molecular_field_exact(const Sym<T>& Qt, const Sym<T>& L, const Coef<T>& c) {
  const Sym<double> Q{double(Qt.xx), double(Qt.xy), double(Qt.xz), double(Qt.yy), double(Qt.yz)};
  const double zz = Q.zz();
  const double sxx = Q.xx * Q.xx + Q.xy * Q.xy + Q.xz * Q.xz;
  const double syy = Q.xy * Q.xy + Q.yy * Q.yy + Q.yz * Q.yz;
  const double szz = Q.xz * Q.xz + Q.yz * Q.yz + zz * zz;
  const double sxy = Q.xx * Q.xy + Q.xy * Q.yy + Q.xz * Q.yz;
  const double sxz = Q.xx * Q.xz + Q.xy * Q.yz + Q.xz * zz;
  const double syz = Q.xy * Q.xz + Q.yy * Q.yz + Q.yz * zz;
  const double tr2 = sxx + syy + szz;
  const double a = c.lin_d - c.quad_d * tr2;
  const double third = c.quad_d * tr2 * (1.0 / 3.0);
  const T bxx = T(a * Q.xx + (c.quad_d * sxx - third)), byy = T(a * Q.yy + (c.quad_d * syy - third));
  const T bxy = T(a * Q.xy + c.quad_d * sxy), bxz = T(a * Q.xz + c.quad_d * sxz), byz = T(a * Q.yz + c.quad_d * syz);
  return Sym<T>{bxx + c.K * L.xx, bxy + c.K * L.xy, bxz + c.K * L.xz, byy + c.K * L.yy, byz + c.K * L.yz};
}

// ---------------------------------------------------------------------------
// Stochastic rounding of the Q update (float form with stochastic
// rounding).  Where the increment of a step is below half a unit in the last
// place of Q (a slowly relaxing bulk, a slowly moving front) round-to-nearest
// drops it at every step and the stored Q stalls; rounding up or down with
// probabilities proportional to the distances keeps the expected stored
// value equal to the exact one.
//
// Counter-based uniform numbers: the PCG hash (the RXS-M-XS output
// permutation of a one-step LCG, O'Neill 2014, used as a hash: Jarzynski
// and Olano, "Hash Functions for GPU Rendering", JCGT 2020) of the site
// index xor a per-step key (itself the hash of the step count).
LC_HD uint32_t pcg_hash(uint32_t v) {
  const uint32_t state = v * 747796405u + 2891336453u;
  const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}

// u * 2^-24, u uniform in (0, 1] from 24 bits of the hash, for site s
// under the step key.
LC_HD float site_uniform(uint32_t s, uint32_t key) {
  const uint32_t h = pcg_hash(s ^ key);
  return float((h >> 8) + 1u) * (1.0f / 281474976710656.0f);
}

// q + inc rounded to float, away from the nearest value with probability
// equal to the distance to it in units in the last place (u24 = u 2^-24,
// u uniform in (0, 1]).  The remainder of the nearest sum is exact when
// |q| >= |inc| (Fast2Sum); where Q is smaller than its increment it is near
// zero and so is its unit in the last place.  For |s| in [2^(ex-1), 2^ex)
// the unit in the last place is 2^(ex-24).
LC_HD float add_stochastic(float q, float inc, float u24) {
  const float s = q + inc;
  const float e = inc - (s - q);
  int ex = 0;
  (void)frexpf(s, &ex);
  const float ulp = ldexpf(1.0f / 16777216.0f, ex);
  return fabsf(e) > ldexpf(u24, ex) ? s + copysignf(ulp, e) : s;
}
LC_HD double add_stochastic(double q, double inc, float) { return q + inc; }

// Stress of Eq. (6) without the hydrostatic part, as a general 3x3 tensor:
//   tau = 2 xi (Q + I/3)(Q:H) - xi [H (Q+I/3) + (Q+I/3) H]
//         - K d_a Q : d_b Q + Q H - H Q.
// With M = H Q this is 2 xi Qp q_h - (2xi/3) H - K E - (xi+1) M - (xi-1) M^T.
// dQ[g] = d_g Q (g = x, y, z).
template <typename T>
LC_HD void stress(const Sym<T>& Q, const Sym<T>& H, const Sym<T> (&dQ)[3],
                                       const Coef<T>& c, T (&tau)[3][3]) {
  const T Qm[3][3] = {{Q.xx, Q.xy, Q.xz}, {Q.xy, Q.yy, Q.yz}, {Q.xz, Q.yz, Q.zz()}};
  const T Hm[3][3] = {{H.xx, H.xy, H.xz}, {H.xy, H.yy, H.yz}, {H.xz, H.yz, H.zz()}};
  const T qh = ddot(Q, H);
  T M[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++)
      M[a][b] = Hm[a][0] * Qm[0][b] + Hm[a][1] * Qm[1][b] + Hm[a][2] * Qm[2][b];
  const T two_xi_qh = T(2) * c.xi * qh;
  const T xi23 = c.xi * T(2.0 / 3.0);
  const T ap = c.xi + T(1), am = c.xi - T(1);
#pragma unroll
  for (int a = 0; a < 3; a++) {
#pragma unroll
    for (int b = 0; b < 3; b++) {
      const T qp = Qm[a][b] + (a == b ? T(1.0 / 3.0) : T(0));
      const T E = ddot(dQ[a], dQ[b]);
      tau[a][b] = two_xi_qh * qp - xi23 * Hm[a][b] - c.K * E - ap * M[a][b] - am * M[b][a];
    }
  }
}

// Column b of the same stress (tau_ab for a = x, y, z), each entry by the
// same expression as in stress(), so bit for bit the same values: what a
// site outside a tile contributes to one derivative of the body force.
template <typename T>
LC_HD void stress_col(const Sym<T>& Q, const Sym<T>& H, const Sym<T> (&dQ)[3], const Coef<T>& c, int b,
                      T (&col)[3]) {
  const T Qm[3][3] = {{Q.xx, Q.xy, Q.xz}, {Q.xy, Q.yy, Q.yz}, {Q.xz, Q.yz, Q.zz()}};
  const T Hm[3][3] = {{H.xx, H.xy, H.xz}, {H.xy, H.yy, H.yz}, {H.xz, H.yz, H.zz()}};
  const T qh = ddot(Q, H);
  const T two_xi_qh = T(2) * c.xi * qh;
  const T xi23 = c.xi * T(2.0 / 3.0);
  const T ap = c.xi + T(1), am = c.xi - T(1);
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const T Mab = Hm[a][0] * Qm[0][b] + Hm[a][1] * Qm[1][b] + Hm[a][2] * Qm[2][b];
    const T Mba = Hm[b][0] * Qm[0][a] + Hm[b][1] * Qm[1][a] + Hm[b][2] * Qm[2][a];
    const T qp = Qm[a][b] + (a == b ? T(1.0 / 3.0) : T(0));
    const T E = ddot(dQ[a], dQ[b]);
    col[a] = two_xi_qh * qp - xi23 * Hm[a][b] - c.K * E - ap * Mab - am * Mba;
  }
}

// Beris-Edwards rate, Eqs. (1)-(2), on the stored components:
//   R = Gamma H + S - (u.grad) Q,
//   S = A + A^T - 2 xi (Q + I/3)(Q:G),  A = [xi D + W](Q + I/3),
// with G[a][b] = d_b u_a, so xi D + W = (xi+1)/2 G + (xi-1)/2 G^T.
// The flow enters through terms that do not depend on Q (Flow): u, the
// matrix B = xi D + W and the five sums g with Q:G = g . (Qxx, Qyy, Qxy,
// Qxz, Qyz) (Qzz = -Qxx - Qyy).  They are formed once per site and serve
// both Heun stages, which use the same u.
// With RAW set, dQ and G are undivided central differences (twice the
// derivatives) and u is halved: the same rate up to rounding (the factors
// of two are exact), with the halvings saved.
template <typename T>
struct Flow {
  T u[3];
  T B[3][3];
  T g[5];
};

template <typename T, bool RAW = false>
LC_HD Flow<T> flow_terms(const T (&u)[3], const T (&G)[3][3], const Coef<T>& c) {
  Flow<T> f;
  const T xp = RAW ? c.xi_p * T(0.5) : c.xi_p, xm = RAW ? c.xi_m * T(0.5) : c.xi_m;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    f.u[a] = u[a];
#pragma unroll
    for (int b = 0; b < 3; b++) f.B[a][b] = xp * G[a][b] + xm * G[b][a];
  }
  f.g[0] = G[0][0] - G[2][2];
  f.g[1] = G[1][1] - G[2][2];
  f.g[2] = G[0][1] + G[1][0];
  f.g[3] = G[0][2] + G[2][0];
  f.g[4] = G[1][2] + G[2][1];
  return f;
}

template <typename T, bool RAW = false>
LC_HD Sym<T> be_rate_flow(const Sym<T>& Q, const Sym<T>& H, const Sym<T> (&dQ)[3], const Flow<T>& f,
                          const Coef<T>& c) {
  const T Qp[3][3] = {{Q.xx + T(1.0 / 3.0), Q.xy, Q.xz},
                      {Q.xy, Q.yy + T(1.0 / 3.0), Q.yz},
                      {Q.xz, Q.yz, Q.zz() + T(1.0 / 3.0)}};
  // S_ab = A_ab + A_ba with A = B Qp.  Each component is accumulated as one
  // chain of fused multiply-adds, starting from the advection term.
  const T qg = Q.xx * f.g[0] + Q.yy * f.g[1] + Q.xy * f.g[2] + Q.xz * f.g[3] + Q.yz * f.g[4];
  const T k = RAW ? c.xi * qg : T(2) * c.xi * qg;
  const T(&u)[3] = f.u;
  // -(u . grad) of one component, then - k Qp_ab
  auto base = [&](T d0, T d1, T d2, T qp) { return -(u[0] * d0) - (u[1] * d1 + (u[2] * d2 + k * qp)); };
  // sum_g B_ag Qp_gb + B_bg Qp_ga added to x
  auto sym = [&](int a, int b, T x) {
    return f.B[a][0] * Qp[0][b] + (f.B[a][1] * Qp[1][b] + (f.B[a][2] * Qp[2][b] +
           (f.B[b][0] * Qp[0][a] + (f.B[b][1] * Qp[1][a] + (f.B[b][2] * Qp[2][a] + x)))));
  };
  // 2 A_aa added to x
  auto diag = [&](int a, T x) {
    return T(2) * (f.B[a][0] * Qp[0][a] + f.B[a][1] * Qp[1][a] + f.B[a][2] * Qp[2][a]) + x;
  };
  Sym<T> R;
  R.xx = c.Gam * H.xx + diag(0, base(dQ[0].xx, dQ[1].xx, dQ[2].xx, Qp[0][0]));
  R.yy = c.Gam * H.yy + diag(1, base(dQ[0].yy, dQ[1].yy, dQ[2].yy, Qp[1][1]));
  R.xy = c.Gam * H.xy + sym(0, 1, base(dQ[0].xy, dQ[1].xy, dQ[2].xy, Qp[0][1]));
  R.xz = c.Gam * H.xz + sym(0, 2, base(dQ[0].xz, dQ[1].xz, dQ[2].xz, Qp[0][2]));
  R.yz = c.Gam * H.yz + sym(1, 2, base(dQ[0].yz, dQ[1].yz, dQ[2].yz, Qp[1][2]));
  return R;
}

template <typename T, bool RAW = false>
LC_HD Sym<T> be_rate(const Sym<T>& Q, const Sym<T>& H, const Sym<T> (&dQ)[3], const T (&u)[3],
                     const T (&G)[3][3], const Coef<T>& c) {
  return be_rate_flow<T, RAW>(Q, H, dQ, flow_terms<T, RAW>(u, G, c), c);
}

// ---------------------------------------------------------------------------
// Periodic neighbour offsets of a site.
struct Nbr {
  int64_t xp, xm, yp, ym, zp, zm;  // index offsets (signed) to the +/- neighbours
};

__device__ __forceinline__ Nbr neighbours(int x, int y, int z, int nx, int ny, int nz) {
  const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
  Nbr n;
  n.xp = (x + 1 == nx) ? -(int64_t)(nx - 1) * sx : sx;
  n.xm = (x == 0) ? (int64_t)(nx - 1) * sx : -sx;
  n.yp = (y + 1 == ny) ? -(int64_t)(ny - 1) * sy : sy;
  n.ym = (y == 0) ? (int64_t)(ny - 1) * sy : -sy;
  n.zp = (z + 1 == nz) ? -(int64_t)(nz - 1) * sz : sz;
  n.zm = (z == 0) ? (int64_t)(nz - 1) * sz : -sz;
  return n;
}

template <typename S>
__device__ __forceinline__ Sym<S> load_sym(const S* __restrict__ q, int64_t N, int64_t s) {
  return Sym<S>{q[s], q[N + s], q[2 * N + s], q[3 * N + s], q[4 * N + s]};
}

template <typename S>
__device__ __forceinline__ void store_sym(S* __restrict__ q, int64_t N, int64_t s, const Sym<S>& v) {
  q[s] = v.xx;
  q[N + s] = v.xy;
  q[2 * N + s] = v.xz;
  q[3 * N + s] = v.yy;
  q[4 * N + s] = v.yz;
}

// Central differences and compact Laplacian of a symmetric tensor field at
// site s (Sec. 1.2.2: second-order differences).
template <typename S, int DIM>
__device__ __forceinline__ void stencil(const S* __restrict__ q, int64_t N, int64_t s, const Nbr& nb,
                                        Sym<S>& c, Sym<S> (&d)[3], Sym<S>& L) {
  c = load_sym(q, N, s);
  const Sym<S> xp = load_sym(q, N, s + nb.xp), xm = load_sym(q, N, s + nb.xm);
  const Sym<S> yp = load_sym(q, N, s + nb.yp), ym = load_sym(q, N, s + nb.ym);
  auto half_diff = [](const Sym<S>& p, const Sym<S>& m) {
    return Sym<S>{(p.xx - m.xx) * S(0.5), (p.xy - m.xy) * S(0.5), (p.xz - m.xz) * S(0.5),
                  (p.yy - m.yy) * S(0.5), (p.yz - m.yz) * S(0.5)};
  };
  d[0] = half_diff(xp, xm);
  d[1] = half_diff(yp, ym);
  L.xx = (xp.xx + xm.xx) + (yp.xx + ym.xx);
  L.xy = (xp.xy + xm.xy) + (yp.xy + ym.xy);
  L.xz = (xp.xz + xm.xz) + (yp.xz + ym.xz);
  L.yy = (xp.yy + xm.yy) + (yp.yy + ym.yy);
  L.yz = (xp.yz + xm.yz) + (yp.yz + ym.yz);
  S ncen = S(-4);
  if constexpr (DIM == 3) {
    const Sym<S> zp = load_sym(q, N, s + nb.zp), zm = load_sym(q, N, s + nb.zm);
    d[2] = half_diff(zp, zm);
    L.xx += zp.xx + zm.xx;
    L.xy += zp.xy + zm.xy;
    L.xz += zp.xz + zm.xz;
    L.yy += zp.yy + zm.yy;
    L.yz += zp.yz + zm.yz;
    ncen = S(-6);
  } else {
    d[2] = sym_zero<S>();
  }
  L.xx += ncen * c.xx;
  L.xy += ncen * c.xy;
  L.xz += ncen * c.xz;
  L.yy += ncen * c.yy;
  L.yz += ncen * c.yz;
}

}  // namespace lc
