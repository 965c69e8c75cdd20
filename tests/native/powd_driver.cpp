// Host build of the library's positive-argument power (csrc/powd.h) for a
// CPU accuracy test: prints the largest relative difference from the C
// library's pow over seeded arguments in the ranges given on the command
// line (log10 x in [lo, hi], y in [ylo, yhi]), and over y = 1 / y.
#define __host__
#define __device__
#define __forceinline__ inline
#include "../../paper_1607_05535_amd/csrc/powd.h"

#include <cstdint>
#include <cstdio>
#include <cstdlib>

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double uniform() {   // SplitMix64 output step, top 53 bits
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}

int main(int argc, char **argv) {
  if (argc != 6) return 2;
  const double lo = atof(argv[1]), hi = atof(argv[2]), ylo = atof(argv[3]), yhi = atof(argv[4]);
  const long n = atol(argv[5]);
  double worst = 0.0, wx = 0.0, wy = 0.0;
  for (long i = 0; i < n; ++i) {
    const double x = std::pow(10.0, lo + (hi - lo) * uniform());
    double y = ylo + (yhi - ylo) * uniform();
    if (i & 1) y = 1.0 / y;
    const double ref = std::pow(x, y), got = thor::powd(x, y);
    const double rel = std::fabs(got - ref) / ref;
    if (rel > worst) { worst = rel; wx = x; wy = y; }
  }
  // exact cases: integer powers of two and x = 1
  double exact = 0.0;
  for (int k = -20; k <= 20; ++k) {
    const double x = std::ldexp(1.0, k);
    exact = std::fmax(exact, std::fabs(thor::powd(x, 2.0) - std::ldexp(1.0, 2 * k)) / std::ldexp(1.0, 2 * k));
  }
  exact = std::fmax(exact, std::fabs(thor::powd(1.0, 1.4) - 1.0));
  printf("%.3e %.17g %.17g %.3e\n", worst, wx, wy, exact);
  return 0;
}
