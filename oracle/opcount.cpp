// opcount.cpp -- TEST INFRASTRUCTURE ONLY.
//
// Floating-point operation count of one time step of the oracle: the
// oracle's own C source (lc_oracle.c), unchanged, compiled as C++ with
// `double` standing for a type that performs every operation in double and
// counts it.  The count is the arithmetic of the method as the oracle
// writes it (full 3x3 tensors, literal index loops, no reuse between
// stages), per site and step; it gives the arithmetic intensity of the
// method against its compulsory bytes.
//
// Build: g++ -O1 -fpermissive -fopenmp oracle/opcount.cpp -o opcount
// Run:   opcount LATTICE N COLL STENCIL   (LATTICE 0 = D2Q9 on N x N,
//        1 = D3Q19 on N^3; COLL 0 = BGK, 1 = MRT; STENCIL 0 = compact,
//        1 = isotropic).  Prints one JSON line with the counts of one step
//        (the difference between runs of one and of zero steps, so that the
//        set-up of the MRT operator is not included) and their sum per site.
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>

namespace opcount {
struct Counts {
  unsigned long long add = 0, mul = 0, div = 0, sqrt = 0, cmp = 0;
};
static Counts g;
}  // namespace opcount

// A double that counts: addition and subtraction, multiplication, division
// and square root are the floating-point operations; comparisons are
// counted apart; negation (a sign flip) is not counted.
struct cd {
  double v;
  cd() = default;
  cd(double x) : v(x) {}
  explicit operator double() const { return v; }
  cd operator-() const { return cd(-v); }
  cd operator+() const { return *this; }
  cd& operator+=(cd b) { opcount::g.add++; v += b.v; return *this; }
  cd& operator-=(cd b) { opcount::g.add++; v -= b.v; return *this; }
  cd& operator*=(cd b) { opcount::g.mul++; v *= b.v; return *this; }
  cd& operator/=(cd b) { opcount::g.div++; v /= b.v; return *this; }
};
static inline cd operator+(cd a, cd b) { opcount::g.add++; return cd(a.v + b.v); }
static inline cd operator-(cd a, cd b) { opcount::g.add++; return cd(a.v - b.v); }
static inline cd operator*(cd a, cd b) { opcount::g.mul++; return cd(a.v * b.v); }
static inline cd operator/(cd a, cd b) { opcount::g.div++; return cd(a.v / b.v); }
static inline bool operator<(cd a, cd b) { opcount::g.cmp++; return a.v < b.v; }
static inline bool operator>(cd a, cd b) { opcount::g.cmp++; return a.v > b.v; }
static inline bool operator<=(cd a, cd b) { opcount::g.cmp++; return a.v <= b.v; }
static inline bool operator>=(cd a, cd b) { opcount::g.cmp++; return a.v >= b.v; }
static inline bool operator==(cd a, cd b) { opcount::g.cmp++; return a.v == b.v; }
static inline bool operator!=(cd a, cd b) { opcount::g.cmp++; return a.v != b.v; }
static inline cd sqrt(cd a) { opcount::g.sqrt++; return cd(std::sqrt(a.v)); }
static inline cd fabs(cd a) { return cd(std::fabs(a.v)); }

#define double cd
#include "lc_oracle.c"
#undef double

static opcount::Counts one_run(int lat, int nx, int ny, int nz, int coll, long steps) {
  const int q = lat == LCO_D2Q9 ? 9 : 19;
  const size_t N = size_t(nx) * ny * nz;
  cd* f = static_cast<cd*>(malloc(q * N * sizeof(cd)));
  cd* q5 = static_cast<cd*>(malloc(5 * N * sizeof(cd)));
  int c[19 * 3];
  cd w[19];
  lco_lattice(lat, c, w);
  // a nonuniform state (the count does not depend on the values: the
  // oracle has no data-dependent arithmetic in a step)
  srand(7);
  for (int i = 0; i < q; i++)
    for (size_t s = 0; s < N; s++) f[i * N + s] = cd(w[i].v * (1.0 + 1e-3 * (rand() / (double)RAND_MAX - 0.5)));
  for (size_t k = 0; k < 5 * N; k++) q5[k] = cd(0.1 * (rand() / (double)RAND_MAX - 0.5));
  const cd p[6] = {cd(1.0), cd(2.7), cd(0.04), cd(0.3), cd(0.7), cd(1.3)};
  cd rates[19];
  for (int k = 0; k < q; k++) rates[k] = cd(1.0 / 1.3);
  opcount::g = opcount::Counts();
  const int rc = coll ? lco_run_coll(lat, nx, ny, nz, p, rates, f, q5, steps) : lco_run(lat, nx, ny, nz, p, f, q5, steps);
  free(f);
  free(q5);
  if (rc != 0) {
    fprintf(stderr, "oracle step failed: %d\n", rc);
    exit(1);
  }
  return opcount::g;
}

int main(int argc, char** argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: %s LATTICE N COLL STENCIL\n", argv[0]);
    return 2;
  }
  const int lat = atoi(argv[1]), n = atoi(argv[2]), coll = atoi(argv[3]), st = atoi(argv[4]);
  if ((lat != 0 && lat != 1) || n < 1 || (coll != 0 && coll != 1) || lco_set_stencil(st) != 0) {
    fprintf(stderr, "bad arguments\n");
    return 2;
  }
  omp_set_num_threads(1);  // one counter
  const int nz = lat == LCO_D2Q9 ? 1 : n;
  const opcount::Counts a = one_run(lat, n, n, nz, coll, 1), b = one_run(lat, n, n, nz, coll, 0);
  const double N = double(n) * n * nz;
  const unsigned long long add = a.add - b.add, mul = a.mul - b.mul, div = a.div - b.div, sq = a.sqrt - b.sqrt;
  printf("{\"lattice\": \"%s\", \"n\": %d, \"collision\": \"%s\", \"stencil\": \"%s\", \"sites\": %.0f, "
         "\"add\": %llu, \"mul\": %llu, \"div\": %llu, \"sqrt\": %llu, \"cmp\": %llu, \"flops_per_site\": %.4f}\n",
         lat ? "D3Q19" : "D2Q9", n, coll ? "mrt" : "bgk", st ? "isotropic" : "compact", N, add, mul, div, sq,
         a.cmp - b.cmp, double(add + mul + div + sq) / N);
  return 0;
}
