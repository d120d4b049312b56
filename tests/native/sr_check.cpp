// Host-side check of the arithmetic of the float form with stochastic
// rounding, compiled from the library's own per-site header:
//  - add_stochastic: exact sums are returned unchanged; otherwise the
//    result is the nearest float or the float one unit in the last place
//    beyond it on the side of the remainder, and its mean over the uniform
//    numbers equals the exact sum (unbiased rounding);
//  - site_uniform: values in (0, 2^-24] with the moments of a uniform
//    distribution;
//  - molecular_field_exact: the bulk part of H (Eq. 4) is the exact value
//    for the float Q, rounded once, also near the nematic minimum where its
//    terms cancel.
// Built and run by tests/test_sr_host.py (CPU only).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "../../paper_1907_13415_amd/csrc/lc_device.h"

using namespace lc;

static int failures = 0;
#define CHECK(cond, ...)                       \
  do {                                         \
    if (!(cond)) {                             \
      std::printf("FAIL %s: ", #cond);         \
      std::printf(__VA_ARGS__);                \
      std::printf("\n");                       \
      failures++;                              \
    }                                          \
  } while (0)

static std::mt19937_64 rng(20190731);
static double urand(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

// spacing of floats just above |s| (s normal)
static double ulp_above(float s) {
  const float a = std::fabs(s);
  return double(std::nextafter(a, INFINITY)) - double(a);
}

// u24 values of site_uniform: k 2^-48, k = 1 .. 2^24; every STRIDE-th one
static constexpr uint32_t STRIDE = 256;
static constexpr uint32_t NU = (1u << 24) / STRIDE;
static float u24_of(uint32_t j) { return float(1u + j * STRIDE) * (1.0f / 281474976710656.0f); }

static void check_pair(float q, float inc) {
  const long double x = (long double)q + (long double)inc;  // exact
  const float s = q + inc;
  const double g = ulp_above(s);
  const long double e = x - (long double)s;
  const float away = e == 0 ? s : float(s + std::copysign(float(g), float(e)));
  long double mean = 0;
  int bad = 0;
  for (uint32_t j = 0; j < NU; j++) {
    const float r = add_stochastic(q, inc, u24_of(j));
    if (r != s && r != away) bad++;
    mean += r;
  }
  mean /= NU;
  CHECK(bad == 0, "q %.9g inc %.9g: %d results outside {nearest, one ulp beyond}", q, inc, bad);
  if (e == 0) {
    CHECK(mean == (long double)s, "q %.9g inc %.9g: exact sum changed", q, inc);
    return;
  }
  // the sampled uniform grid has spacing STRIDE 2^-24: the mean is the
  // exact sum to that fraction of a unit in the last place
  const long double tol = (long double)g * (2.0L * STRIDE / 16777216.0L);
  CHECK(std::fabs((double)(mean - x)) <= (double)tol, "q %.9g inc %.9g: mean off by %.3e ulp", q, inc,
        (double)((mean - x) / (long double)g));
}

static void check_add_stochastic() {
  int n = 0;
  // random magnitudes and signs: increments from 1e-10 to 1e-1 of Q
  for (int t = 0; t < 400; t++, n++) {
    const float q = float(urand(-1.0, 1.0));
    const float inc = float(q * std::pow(10.0, urand(-10.0, -1.0)) * (urand(0, 1) < 0.5 ? -1 : 1));
    check_pair(q, inc);
  }
  // below half a unit in the last place: round-to-nearest would stall
  for (int t = 0; t < 100; t++, n++) {
    const float q = float(urand(0.1, 0.9));
    check_pair(q, float(urand(-0.49, 0.49) * ulp_above(q)));
  }
  // powers of two, with remainders towards and away from zero
  for (int k = -6; k <= 0; k++)
    for (double f : {-0.7, -0.3, -1e-3, 1e-3, 0.3, 0.7}) {
      const float q = std::ldexp(1.0f, k);
      check_pair(q, float(f * ulp_above(q)));
      check_pair(-q, float(-f * ulp_above(q)));
      n += 2;
    }
  // exact sums and zero
  check_pair(0.5f, 0.25f);
  check_pair(0.0f, 1e-9f);
  check_pair(0.3f, 0.0f);
  n += 3;
  // a stalled relaxation: 1000 increments of 0.1 ulp move Q by 100 ulp on
  // average (round-to-nearest would not move it)
  {
    const float q0 = 0.4f;
    const float inc = float(0.1 * ulp_above(q0));
    double total = 0;
    const int runs = 64;
    for (int r = 0; r < runs; r++) {
      float q = q0;
      for (int i = 0; i < 1000; i++) q = add_stochastic(q, inc, site_uniform(uint32_t(i), pcg_hash(uint32_t(r))));
      total += (double(q) - double(q0)) / ulp_above(q0);
    }
    const double moved = total / runs;
    CHECK(std::fabs(moved - 100.0) < 5.0, "1000 steps of 0.1 ulp moved Q by %.2f ulp on average", moved);
    std::printf("stalled relaxation: mean move %.2f ulp (expected 100)\n", moved);
  }
  std::printf("add_stochastic: %d cases, %u uniform numbers each\n", n, NU);
}

static void check_site_uniform() {
  const uint32_t n = 1u << 22;
  for (uint32_t key : {0u, pcg_hash(1u), pcg_hash(12345u)}) {
    double m1 = 0, m2 = 0;
    float lo = 1, hi = 0;
    uint32_t dec[10] = {0};
    for (uint32_t s = 0; s < n; s++) {
      const double u = double(site_uniform(s, key)) * 16777216.0;  // in (0, 1]
      m1 += u;
      m2 += u * u;
      lo = std::fmin(lo, float(u));
      hi = std::fmax(hi, float(u));
      dec[std::min(9, int(u * 10))]++;
    }
    m1 /= n;
    m2 /= n;
    CHECK(lo > 0 && hi <= 1, "key %u: range [%g, %g]", key, lo, hi);
    CHECK(std::fabs(m1 - 0.5) < 2e-3, "key %u: mean %.5f", key, m1);
    CHECK(std::fabs(m2 - 1.0 / 3.0) < 2e-3, "key %u: second moment %.5f", key, m2);
    for (int d = 0; d < 10; d++)
      CHECK(std::fabs(double(dec[d]) / n - 0.1) < 2e-3, "key %u: decile %d holds %.4f", key, d, double(dec[d]) / n);
  }
  // two step keys give uncorrelated numbers at the same sites
  double c = 0;
  for (uint32_t s = 0; s < n; s++)
    c += (double(site_uniform(s, pcg_hash(7u))) * 16777216.0 - 0.5) *
         (double(site_uniform(s, pcg_hash(8u))) * 16777216.0 - 0.5);
  c = c / n * 12.0;
  CHECK(std::fabs(c) < 5e-3, "correlation of two step keys %.4f", c);
  std::printf("site_uniform: 3 keys x %u sites, correlation of two keys %.2e\n", n, c);
}

static Coef<float> coefs(double gamma, double K) {
  Coef<float> c{};
  const double A0 = 1.0;
  c.lin_d = -A0 * (1.0 - gamma / 3.0);
  c.quad_d = A0 * gamma;
  c.lin = float(c.lin_d);
  c.quad = float(c.quad_d);
  c.K = float(K);
  return c;
}

// bulk part of Eq. (4) in long double: lin Q + quad (Q.Q - tr(Q.Q) I/3) - quad tr(Q.Q) Q
static void bulk_exact(const Sym<float>& Qf, double lin, double quad, long double (&h)[5]) {
  const long double Q[3][3] = {{Qf.xx, Qf.xy, Qf.xz}, {Qf.xy, Qf.yy, Qf.yz},
                               {Qf.xz, Qf.yz, -(long double)Qf.xx - (long double)Qf.yy}};
  long double QQ[3][3], tr = 0;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      QQ[a][b] = 0;
      for (int g = 0; g < 3; g++) QQ[a][b] += Q[a][g] * Q[g][b];
    }
  for (int a = 0; a < 3; a++) tr += QQ[a][a];
  auto H = [&](int a, int b) {
    return (long double)lin * Q[a][b] + (long double)quad * (QQ[a][b] - (a == b ? tr / 3 : 0)) -
           (long double)quad * tr * Q[a][b];
  };
  h[0] = H(0, 0);
  h[1] = H(0, 1);
  h[2] = H(0, 2);
  h[3] = H(1, 1);
  h[4] = H(1, 2);
}

static float comp(const Sym<float>& s, int k) {
  return k == 0 ? s.xx : k == 1 ? s.xy : k == 2 ? s.xz : k == 3 ? s.yy : s.yz;
}

static void check_molecular_field() {
  const Sym<float> L0{0, 0, 0, 0, 0};
  double worst_exact = 0, worst_plain = 0;   // at the nematic minimum
  double worst_exact_any = 0;
  for (double gamma : {2.7, 2.705, 3.0}) {
    const Coef<float> c = coefs(gamma, 0.04);
    const double Sn = 0.25 + 0.75 * std::sqrt(1.0 - 8.0 / (3.0 * gamma));
    for (int t = 0; t < 2000; t++) {
      Sym<float> Q;
      if (t % 2 == 0) {  // random tensor
        Q = Sym<float>{float(urand(-0.3, 0.3)), float(urand(-0.3, 0.3)), float(urand(-0.3, 0.3)),
                       float(urand(-0.3, 0.3)), float(urand(-0.3, 0.3))};
      } else {  // the uniaxial nematic minimum along a random director
        double n[3] = {urand(-1, 1), urand(-1, 1), urand(-1, 1)};
        const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (double& v : n) v /= nn;
        Q = Sym<float>{float(Sn * (n[0] * n[0] - 1.0 / 3)), float(Sn * n[0] * n[1]), float(Sn * n[0] * n[2]),
                       float(Sn * (n[1] * n[1] - 1.0 / 3)), float(Sn * n[1] * n[2])};
      }
      long double h[5];
      bulk_exact(Q, c.lin_d, c.quad_d, h);
      const Sym<float> He = molecular_field_exact(Q, L0, c);
      const Sym<float> Hp = molecular_field(Q, L0, c);
      for (int k = 0; k < 5; k++) {
        const float v = comp(He, k);
        // one rounding of the exact value (double sum: a few units of 2^-53
        // relative to the largest term on top)
        const double half_ulp = 0.5 * ulp_above(float(h[k])) + 1e-15;
        const double err = std::fabs((double)((long double)v - h[k]));
        CHECK(err <= half_ulp, "gamma %g case %d comp %d: |H - exact| = %.3e > %.3e", gamma, t, k, err, half_ulp);
        worst_exact_any = std::fmax(worst_exact_any, err);
        if (t % 2) {
          worst_exact = std::fmax(worst_exact, err);
          worst_plain = std::fmax(worst_plain, std::fabs((double)((long double)comp(Hp, k) - h[k])));
        }
      }
      // the gradient term is added in float to the rounded bulk part
      const Sym<float> L{float(urand(-1, 1)), float(urand(-1, 1)), float(urand(-1, 1)), float(urand(-1, 1)),
                         float(urand(-1, 1))};
      const Sym<float> HL = molecular_field_exact(Q, L, c);
      for (int k = 0; k < 5; k++) {
        const double kl = double(c.K) * double(comp(L, k));
        const double want = double(comp(He, k)) + kl;
        CHECK(std::fabs(double(comp(HL, k)) - want) <= ulp_above(float(want)) + ulp_above(float(kl)),
              "gamma %g case %d comp %d: K L not added in float", gamma, t, k);
      }
    }
  }
  std::printf("molecular field, bulk part: worst error %.3e over all cases; at the nematic minimum %.3e "
              "(double sum) against %.3e (float sum)\n", worst_exact_any, worst_exact, worst_plain);
  // at the nematic minimum the float sum leaves errors far above those of
  // the double sum, which is why the double sum is used
  CHECK(worst_plain > 1000 * worst_exact, "float sum not worse than double sum (%.3e vs %.3e)", worst_plain,
        worst_exact);
}

int main() {
  check_add_stochastic();
  check_site_uniform();
  check_molecular_field();
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "OK", failures);
  return failures ? 1 : 0;
}
