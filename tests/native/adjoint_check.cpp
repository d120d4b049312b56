// Host-side check of the per-site reverse-mode functions of the HIP
// library: every vector-Jacobian product is compared with central finite
// differences of the corresponding forward function, in double precision,
// on random inputs.  Built and run by tests/test_adjoint_host.py (CPU only).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "../../paper_1907_13415_amd/csrc/lc_adjoint.h"

using namespace lc;
using T = double;

static std::mt19937_64 rng(12345);
static T rnd(T a = 1.0) { return std::uniform_real_distribution<T>(-a, a)(rng); }
static Sym<T> rsym(T a) { return Sym<T>{rnd(a), rnd(a), rnd(a), rnd(a), rnd(a)}; }
static T* comp(Sym<T>& s, int k) { return k == 0 ? &s.xx : k == 1 ? &s.xy : k == 2 ? &s.xz : k == 3 ? &s.yy : &s.yz; }

static Coef<T> coefs() {
  Coef<T> c;
  const T A0 = 0.9, g = 2.73, K = 0.07, Gam = 0.31, xi = 0.7, tau = 1.3;
  c.lin = -A0 * (1 - g / 3);
  c.quad = A0 * g;
  c.K = K;
  c.Gam = Gam;
  c.xi = xi;
  c.xi_p = (xi + 1) / 2;
  c.xi_m = (xi - 1) / 2;
  c.omega = 1 / tau;
  c.src = 1 - 1 / (2 * tau);
  c.A0 = A0;
  return c;
}
static Coef<T> with(const Coef<T>& c0, int which, T delta) {
  // which: 0 gamma, 1 K, 2 Gamma
  Coef<T> c = c0;
  if (which == 0) {
    c.lin += c.A0 * delta / 3;
    c.quad += c.A0 * delta;
  } else if (which == 1) {
    c.K += delta;
  } else {
    c.Gam += delta;
  }
  return c;
}

static double worst = 0;
static void check(const char* what, T got, T want, T scale) {
  const T e = std::fabs(got - want) / std::fmax(std::fabs(want), scale);
  if (e > worst) worst = e;
  if (e > 1e-6) std::printf("MISMATCH %s: vjp %.12e fd %.12e\n", what, got, want);
}

int main() {
  const T h = 1e-6;
  const Coef<T> c = coefs();
  for (int trial = 0; trial < 20; trial++) {
    // ---- molecular field
    {
      Sym<T> Q = rsym(0.3), L = rsym(0.1), Hb = rsym(1.0);
      auto phi = [&](const Sym<T>& q, const Sym<T>& l, const Coef<T>& cc) { return dot5(Hb, molecular_field(q, l, cc)); };
      Sym<T> Qb = sym_zero<T>(), Lb;
      T d[3] = {0, 0, 0};
      molecular_field_vjp(Q, L, Hb, c, Qb, Lb, d);
      for (int k = 0; k < 5; k++) {
        Sym<T> qp = Q, qm = Q, lp = L, lm = L;
        *comp(qp, k) += h;
        *comp(qm, k) -= h;
        *comp(lp, k) += h;
        *comp(lm, k) -= h;
        check("H/dQ", *comp(Qb, k), (phi(qp, L, c) - phi(qm, L, c)) / (2 * h), 1e-3);
        check("H/dL", *comp(Lb, k), (phi(Q, lp, c) - phi(Q, lm, c)) / (2 * h), 1e-3);
      }
      for (int w = 0; w < 2; w++)
        check("H/dparam", d[w], (phi(Q, L, with(c, w, h)) - phi(Q, L, with(c, w, -h))) / (2 * h), 1e-3);
    }
    // ---- stress
    {
      Sym<T> Q = rsym(0.3), H = rsym(0.2), dQ[3] = {rsym(0.1), rsym(0.1), rsym(0.1)};
      T tb[3][3];
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) tb[a][b] = rnd();
      auto phi = [&](const Sym<T>& q, const Sym<T>& hh, const Sym<T> (&dq)[3], const Coef<T>& cc) {
        T t[3][3];
        stress(q, hh, dq, cc, t);
        T s = 0;
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) s += tb[a][b] * t[a][b];
        return s;
      };
      Sym<T> Qb = sym_zero<T>(), Hb = sym_zero<T>(), dQb[3] = {sym_zero<T>(), sym_zero<T>(), sym_zero<T>()};
      T d[3] = {0, 0, 0};
      stress_vjp(Q, H, dQ, tb, c, Qb, Hb, dQb, d);
      for (int k = 0; k < 5; k++) {
        Sym<T> qp = Q, qm = Q, hp = H, hm = H;
        *comp(qp, k) += h;
        *comp(qm, k) -= h;
        *comp(hp, k) += h;
        *comp(hm, k) -= h;
        check("tau/dQ", *comp(Qb, k), (phi(qp, H, dQ, c) - phi(qm, H, dQ, c)) / (2 * h), 1e-3);
        check("tau/dH", *comp(Hb, k), (phi(Q, hp, dQ, c) - phi(Q, hm, dQ, c)) / (2 * h), 1e-3);
        for (int g = 0; g < 3; g++) {
          Sym<T> dp[3] = {dQ[0], dQ[1], dQ[2]}, dm[3] = {dQ[0], dQ[1], dQ[2]};
          *comp(dp[g], k) += h;
          *comp(dm[g], k) -= h;
          check("tau/ddQ", *comp(dQb[g], k), (phi(Q, H, dp, c) - phi(Q, H, dm, c)) / (2 * h), 1e-3);
        }
      }
      check("tau/dK", d[1], (phi(Q, H, dQ, with(c, 1, h)) - phi(Q, H, dQ, with(c, 1, -h))) / (2 * h), 1e-3);
    }
    // ---- Beris-Edwards rate
    {
      Sym<T> Q = rsym(0.3), H = rsym(0.2), dQ[3] = {rsym(0.1), rsym(0.1), rsym(0.1)}, Rb = rsym(1.0);
      T u[3] = {rnd(0.05), rnd(0.05), rnd(0.05)}, G[3][3];
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G[a][b] = rnd(0.02);
      auto phi = [&](const Sym<T>& q, const Sym<T>& hh, const Sym<T> (&dq)[3], const T (&uu)[3], const T (&gg)[3][3],
                     const Coef<T>& cc) { return dot5(Rb, be_rate(q, hh, dq, uu, gg, cc)); };
      Sym<T> Qb = sym_zero<T>(), Hb = sym_zero<T>(), dQb[3] = {sym_zero<T>(), sym_zero<T>(), sym_zero<T>()};
      T ub[3] = {0, 0, 0}, Gb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, d[3] = {0, 0, 0};
      be_rate_vjp(Q, H, dQ, u, G, Rb, c, Qb, Hb, dQb, ub, Gb, d);
      for (int k = 0; k < 5; k++) {
        Sym<T> qp = Q, qm = Q, hp = H, hm = H;
        *comp(qp, k) += h;
        *comp(qm, k) -= h;
        *comp(hp, k) += h;
        *comp(hm, k) -= h;
        check("R/dQ", *comp(Qb, k), (phi(qp, H, dQ, u, G, c) - phi(qm, H, dQ, u, G, c)) / (2 * h), 1e-3);
        check("R/dH", *comp(Hb, k), (phi(Q, hp, dQ, u, G, c) - phi(Q, hm, dQ, u, G, c)) / (2 * h), 1e-3);
        for (int g = 0; g < 3; g++) {
          Sym<T> dp[3] = {dQ[0], dQ[1], dQ[2]}, dm[3] = {dQ[0], dQ[1], dQ[2]};
          *comp(dp[g], k) += h;
          *comp(dm[g], k) -= h;
          check("R/ddQ", *comp(dQb[g], k), (phi(Q, H, dp, u, G, c) - phi(Q, H, dm, u, G, c)) / (2 * h), 1e-3);
        }
      }
      for (int a = 0; a < 3; a++) {
        T up[3] = {u[0], u[1], u[2]}, um[3] = {u[0], u[1], u[2]};
        up[a] += h;
        um[a] -= h;
        check("R/du", ub[a], (phi(Q, H, dQ, up, G, c) - phi(Q, H, dQ, um, G, c)) / (2 * h), 1e-3);
        for (int b = 0; b < 3; b++) {
          T gp[3][3], gm[3][3];
          for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) gp[i][j] = gm[i][j] = G[i][j];
          gp[a][b] += h;
          gm[a][b] -= h;
          check("R/dG", Gb[a][b], (phi(Q, H, dQ, u, gp, c) - phi(Q, H, dQ, u, gm, c)) / (2 * h), 1e-3);
        }
      }
      check("R/dGamma", d[2], (phi(Q, H, dQ, u, G, with(c, 2, h)) - phi(Q, H, dQ, u, G, with(c, 2, -h))) / (2 * h),
            1e-3);
    }
    // ---- collision (D2Q9 and D3Q19)
    auto coll = [&](auto lat_tag) {
      constexpr int LAT = decltype(lat_tag)::value;
      using Lt = Lattice<LAT>;
      T f[Lt::q], fbs[Lt::q];
      for (int i = 0; i < Lt::q; i++) {
        f[i] = Lt::w(i) * (1 + rnd(0.01));
        fbs[i] = rnd();
      }
      T rho = 1 + rnd(0.01), u[3] = {rnd(0.05), rnd(0.05), LAT == 1 ? rnd(0.05) : 0.0},
        F[3] = {rnd(0.01), rnd(0.01), LAT == 1 ? rnd(0.01) : 0.0};
      auto phi = [&](const T (&ff)[Lt::q], T r, const T (&uu)[3], const T (&FF)[3]) {
        T s = 0;
        const T uu2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
        for (int i = 0; i < Lt::q; i++) {
          const T w = Lt::w(i), cu = Lt::cx(i) * uu[0] + Lt::cy(i) * uu[1] + Lt::cz(i) * uu[2];
          const T cF = Lt::cx(i) * FF[0] + Lt::cy(i) * FF[1] + Lt::cz(i) * FF[2];
          const T uF = uu[0] * FF[0] + uu[1] * FF[1] + uu[2] * FF[2];
          const T feq = w * r * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu2);
          const T src = w * c.src * (3 * cF * (1 + 3 * cu) - 3 * uF);
          s += fbs[i] * ((1 - c.omega) * ff[i] + c.omega * feq + src);
        }
        return s;
      };
      T fb[Lt::q] = {}, rb = 0, ub[3] = {0, 0, 0}, Fb[3] = {0, 0, 0};
      collide_vjp<LAT, T>(fbs, rho, u, F, c, fb, rb, ub, Fb);
      for (int i = 0; i < Lt::q; i++) {
        T fp[Lt::q], fm[Lt::q];
        for (int j = 0; j < Lt::q; j++) fp[j] = fm[j] = f[j];
        fp[i] += h;
        fm[i] -= h;
        check("C/df", fb[i], (phi(fp, rho, u, F) - phi(fm, rho, u, F)) / (2 * h), 1e-3);
      }
      check("C/drho", rb, (phi(f, rho + h, u, F) - phi(f, rho - h, u, F)) / (2 * h), 1e-3);
      for (int a = 0; a < 3; a++) {
        T up[3] = {u[0], u[1], u[2]}, um[3] = {u[0], u[1], u[2]}, Fp[3] = {F[0], F[1], F[2]}, Fm[3] = {F[0], F[1], F[2]};
        up[a] += h;
        um[a] -= h;
        Fp[a] += h;
        Fm[a] -= h;
        check("C/du", ub[a], (phi(f, rho, up, F) - phi(f, rho, um, F)) / (2 * h), 1e-3);
        check("C/dF", Fb[a], (phi(f, rho, u, Fp) - phi(f, rho, u, Fm)) / (2 * h), 1e-3);
      }
    };
    coll(std::integral_constant<int, 0>());
    coll(std::integral_constant<int, 1>());
  }
  std::printf("worst relative error %.3e\n", worst);
  return worst < 1e-7 ? 0 : 1;
}
