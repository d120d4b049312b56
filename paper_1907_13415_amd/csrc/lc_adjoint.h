// lc_adjoint.h -- reverse-mode (vector-Jacobian) forms of the per-site
// functions of one step.
//
// Each *_vjp takes the forward inputs and the adjoint of the outputs and
// accumulates (+=) the adjoints of the inputs.  Symmetric traceless inputs
// are the five stored components, so the adjoint of the full tensor Qm is
// mapped back by sym_adj (Qzz = -Qxx - Qyy, off-diagonals counted twice);
// outputs that are the stored components of a full tensor are embedded by
// embed5.  Parameter derivatives (gamma, K, Gamma) accumulate into d[3].
#pragma once

#include "lc_device.h"

namespace lc {

template <typename T>
LC_HD void full3(const Sym<T>& a, T (&m)[3][3]) {
  m[0][0] = a.xx;
  m[0][1] = a.xy;
  m[0][2] = a.xz;
  m[1][0] = a.xy;
  m[1][1] = a.yy;
  m[1][2] = a.yz;
  m[2][0] = a.xz;
  m[2][1] = a.yz;
  m[2][2] = -a.xx - a.yy;
}

// adjoint of Sym -> full tensor
template <typename T>
LC_HD Sym<T> sym_adj(const T (&g)[3][3]) {
  return Sym<T>{g[0][0] - g[2][2], g[0][1] + g[1][0], g[0][2] + g[2][0], g[1][1] - g[2][2], g[1][2] + g[2][1]};
}

// adjoint of taking the five stored components of a full tensor
template <typename T>
LC_HD void embed5(const Sym<T>& a, T (&m)[3][3]) {
  m[0][0] = a.xx;
  m[0][1] = a.xy;
  m[0][2] = a.xz;
  m[1][0] = T(0);
  m[1][1] = a.yy;
  m[1][2] = a.yz;
  m[2][0] = T(0);
  m[2][1] = T(0);
  m[2][2] = T(0);
}

template <typename T>
LC_HD T dot5(const Sym<T>& a, const Sym<T>& b) {
  return a.xx * b.xx + a.xy * b.xy + a.xz * b.xz + a.yy * b.yy + a.yz * b.yz;
}

template <typename T>
LC_HD void add_to(Sym<T>& a, const Sym<T>& b) {
  a.xx += b.xx;
  a.xy += b.xy;
  a.xz += b.xz;
  a.yy += b.yy;
  a.yz += b.yz;
}

// d = (d_gamma, d_K, d_Gamma)
// Molecular field H(Q, L) of Eq. (4):
//   H = lin Q + quad (Q.Q - tr2 I/3) - quad tr2 Q + K L,
//   lin = -A0 (1 - gamma/3), quad = A0 gamma, tr2 = Q:Q.
template <typename T>
LC_HD void molecular_field_vjp(const Sym<T>& Q, const Sym<T>& L, const Sym<T>& Hb, const Coef<T>& c, Sym<T>& Qb,
                               Sym<T>& Lb, T (&d)[3]) {
  T Qm[3][3], Hm[3][3];
  full3(Q, Qm);
  embed5(Hb, Hm);
  T tr2 = T(0), qh = T(0);
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      tr2 += Qm[a][b] * Qm[a][b];
      qh += Qm[a][b] * Hm[a][b];
    }
  const T trH = Hm[0][0] + Hm[1][1] + Hm[2][2];
  T g[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      T hq = T(0), qhm = T(0);
#pragma unroll
      for (int k = 0; k < 3; k++) {
        hq += Hm[a][k] * Qm[k][b];
        qhm += Qm[a][k] * Hm[k][b];
      }
      g[a][b] = (c.lin - c.quad * tr2) * Hm[a][b] + c.quad * (hq + qhm) -
                c.quad * (T(2.0 / 3.0) * trH + T(2) * qh) * Qm[a][b];
    }
  add_to(Qb, sym_adj(g));
  Lb = Sym<T>{c.K * Hb.xx, c.K * Hb.xy, c.K * Hb.xz, c.K * Hb.yy, c.K * Hb.yz};
  // dH/dgamma = (A0/3) Q + A0 (Q.Q - tr2 I/3 - tr2 Q)
  T QQ[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) QQ[a][b] = Qm[a][0] * Qm[0][b] + Qm[a][1] * Qm[1][b] + Qm[a][2] * Qm[2][b];
  auto dHg = [&](int a, int b) {
    return c.A0 * (Qm[a][b] * T(1.0 / 3.0) + QQ[a][b] - (a == b ? tr2 * T(1.0 / 3.0) : T(0)) - tr2 * Qm[a][b]);
  };
  d[0] += Hb.xx * dHg(0, 0) + Hb.xy * dHg(0, 1) + Hb.xz * dHg(0, 2) + Hb.yy * dHg(1, 1) + Hb.yz * dHg(1, 2);
  d[1] += dot5(Hb, L);
}

// Stress of Eq. (6) (see stress()):
//   tau = 2 xi qh (Q + I/3) - (2 xi/3) H - K E - (xi+1) M - (xi-1) M^T,
//   M = H Q, qh = Q:H, E_ab = d_a Q : d_b Q.
template <typename T>
LC_HD void stress_vjp(const Sym<T>& Q, const Sym<T>& H, const Sym<T> (&dQ)[3], const T (&tb)[3][3],
                      const Coef<T>& c, Sym<T>& Qb, Sym<T>& Hb, Sym<T> (&dQb)[3], T (&d)[3]) {
  T Qm[3][3], Hm[3][3];
  full3(Q, Qm);
  full3(H, Hm);
  T qh = T(0), qbar = T(0);
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      qh += Qm[a][b] * Hm[a][b];
      qbar += tb[a][b] * (Qm[a][b] + (a == b ? T(1.0 / 3.0) : T(0)));
    }
  qbar *= T(2) * c.xi;
  const T ap = c.xi + T(1), am = c.xi - T(1);
  T Mb[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) Mb[a][b] = -ap * tb[a][b] - am * tb[b][a];
  T gQ[3][3], gH[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      T mq = T(0), hm = T(0);
#pragma unroll
      for (int k = 0; k < 3; k++) {
        mq += Mb[a][k] * Qm[b][k];  // (Mb Q^T)_ab, M = H Q
        hm += Hm[k][a] * Mb[k][b];  // (H^T Mb)_ab
      }
      gQ[a][b] = T(2) * c.xi * qh * tb[a][b] + hm + qbar * Hm[a][b];
      gH[a][b] = -(T(2) * c.xi / T(3)) * tb[a][b] + mq + qbar * Qm[a][b];
    }
  add_to(Qb, sym_adj(gQ));
  add_to(Hb, sym_adj(gH));
  // elastic part: E_ab = sum_{gn} dQ_a[gn] dQ_b[gn]
  T D[3][3][3];
#pragma unroll
  for (int a = 0; a < 3; a++) full3(dQ[a], D[a]);
  T Eb[3][3];
  T dk = T(0);
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      Eb[a][b] = -c.K * tb[a][b];
      dk -= tb[a][b] * ddot(dQ[a], dQ[b]);
    }
  d[1] += dk;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    T g[3][3];
#pragma unroll
    for (int p = 0; p < 3; p++)
#pragma unroll
      for (int q = 0; q < 3; q++) {
        T acc = T(0);
#pragma unroll
        for (int b = 0; b < 3; b++) acc += (Eb[a][b] + Eb[b][a]) * D[b][p][q];
        g[p][q] = acc;
      }
    add_to(dQb[a], sym_adj(g));
  }
}

// Beris-Edwards rate on the stored components (see be_rate()):
//   R = Gamma H + P5(A + A^T - k (Q + I/3)) - u.grad Q,
//   A = B (Q + I/3), B = xi_p G + xi_m G^T, k = 2 xi (Q:G).
template <typename T>
LC_HD void be_rate_vjp(const Sym<T>& Q, const Sym<T>& H, const Sym<T> (&dQ)[3], const T (&u)[3],
                       const T (&G)[3][3], const Sym<T>& Rb, const Coef<T>& c, Sym<T>& Qb, Sym<T>& Hb,
                       Sym<T> (&dQb)[3], T (&ub)[3], T (&Gb)[3][3], T (&d)[3]) {
  d[2] += dot5(Rb, H);
  add_to(Hb, Sym<T>{c.Gam * Rb.xx, c.Gam * Rb.xy, c.Gam * Rb.xz, c.Gam * Rb.yy, c.Gam * Rb.yz});
#pragma unroll
  for (int g = 0; g < 3; g++) {
    ub[g] -= dot5(Rb, dQ[g]);
    add_to(dQb[g], Sym<T>{-u[g] * Rb.xx, -u[g] * Rb.xy, -u[g] * Rb.xz, -u[g] * Rb.yy, -u[g] * Rb.yz});
  }
  T Qm[3][3], Rm[3][3];
  full3(Q, Qm);
  embed5(Rb, Rm);
  T Qp[3][3], B[3][3];
  T qg = T(0), kb = T(0);
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      Qp[a][b] = Qm[a][b] + (a == b ? T(1.0 / 3.0) : T(0));
      B[a][b] = c.xi_p * G[a][b] + c.xi_m * G[b][a];
      qg += Qm[a][b] * G[a][b];
    }
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) kb -= Rm[a][b] * Qp[a][b];
  const T k = T(2) * c.xi * qg;
  const T qgb = T(2) * c.xi * kb;
  T Ab[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) Ab[a][b] = Rm[a][b] + Rm[b][a];
  T gQ[3][3], Bb[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      T bq = T(0), ba = T(0);
#pragma unroll
      for (int m = 0; m < 3; m++) {
        bq += Ab[a][m] * Qp[b][m];  // (Ab Qp^T)_ab
        ba += B[m][a] * Ab[m][b];   // (B^T Ab)_ab
      }
      Bb[a][b] = bq;
      gQ[a][b] = -k * Rm[a][b] + ba + qgb * G[a][b];
    }
  add_to(Qb, sym_adj(gQ));
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) Gb[a][b] += c.xi_p * Bb[a][b] + c.xi_m * Bb[b][a] + qgb * Qm[a][b];
}

// BGK collision with forcing for one site, logical populations (no
// deviation form): f* = (1 - omega) f + omega f_eq(rho, u) + S(u, F).
template <int LAT, typename T>
LC_HD void collide_vjp(const T (&fb_star)[Lattice<LAT>::q], T rho, const T (&u)[3], const T (&F)[3], const Coef<T>& c,
                       T (&fb)[Lattice<LAT>::q], T& rhob, T (&ub)[3], T (&Fb)[3]) {
  using L = Lattice<LAT>;
  const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int i = 0; i < L::q; i++) {
    const T w = T(L::w(i));
    const T cx = T(L::cx(i)), cy = T(L::cy(i)), cz = T(L::cz(i));
    const T cu = cx * u[0] + cy * u[1] + cz * u[2];
    const T cF = cx * F[0] + cy * F[1] + cz * F[2];
    const T a = fb_star[i];
    fb[i] += (T(1) - c.omega) * a;
    rhob += a * c.omega * w * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu);
    const T cc[3] = {cx, cy, cz};
#pragma unroll
    for (int al = 0; al < 3; al++) {
      ub[al] += a * (c.omega * w * rho * (T(3) * cc[al] + T(9) * cu * cc[al] - T(3) * u[al]) +
                     w * c.src * (T(9) * cF * cc[al] - T(3) * F[al]));
      Fb[al] += a * w * c.src * (T(3) * cc[al] * (T(1) + T(3) * cu) - T(3) * u[al]);
    }
  }
}

}  // namespace lc
