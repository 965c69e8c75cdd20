// Drives the host grid builder through its C entry points for a range of
// grid levels, standard and smoothed, and through its argument checks; built
// with AddressSanitizer and UndefinedBehaviorSanitizer by the test beside it.
// The error-message sink of the library's runtime is stubbed here.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/thor.h"

namespace thor {
void set_error(const std::string &) {}
void clear_error() {}
}  // namespace thor

int main() {
  for (int g = 0; g <= 4; ++g)
    for (int smooth = 0; smooth <= 1; ++smooth) {
      thor_grid_params p;
      thor_grid_params_default(g, &p);
      p.smooth = smooth;
      thor_grid *grid = nullptr;
      const int rc = thor_grid_build(&p, &grid);
      if (rc != THOR_OK || !grid) { std::printf("build g%d smooth %d: %d\n", g, smooth, rc); return 1; }
      int64_t n = 0;
      int npent = 0, iters = 0;
      thor_grid_info(grid, &n, &npent, &iters);
      if (n != 10 * (int64_t(1) << (2 * g)) + 2 || npent != 12) { std::printf("counts g%d\n", g); return 1; }
      std::vector<int32_t> nbr(n * 6), idx(n * 18);
      std::vector<double> xyz(n * 3), area(n), dc(n * 21), lc(n * 6), w(n * 54);
      if (thor_grid_export(grid, nbr.data(), xyz.data(), area.data()) != THOR_OK ||
          thor_grid_coefficients(grid, dc.data(), lc.data()) != THOR_OK ||
          thor_grid_damping_coefficients(grid, idx.data(), w.data()) != THOR_OK ||
          thor_grid_export(grid, nullptr, nullptr, nullptr) != THOR_OK) {
        std::printf("export g%d\n", g);
        return 1;
      }
      thor_grid_free(grid);
    }
  // argument errors
  thor_grid_params p;
  thor_grid_params_default(3, &p);
  p.glevel = 9;
  thor_grid *grid = nullptr;
  if (thor_grid_build(&p, &grid) != THOR_EINVAL) return 1;
  if (thor_grid_build(nullptr, &grid) != THOR_EINVAL) return 1;
  thor_grid_params_default(3, &p);
  p.max_iter = 3;
  if (thor_grid_build(&p, &grid) != THOR_ENOTCONV || !grid) return 1;
  thor_grid_free(grid);
  std::printf("ok\n");
  return 0;
}
