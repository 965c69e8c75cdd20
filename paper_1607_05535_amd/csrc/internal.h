// Internal declarations shared by the host sources of libthor.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/thor.h"

namespace thor {

constexpr int kRing2 = 18;   // columns of the two-ring around a column, at most

struct Vec3 {
  double x, y, z;
};

// Host-side grid: topology, unit-sphere geometry and operator coefficients.
struct Grid {
  int glevel = 0;
  int smooth = 1;
  int64_t n = 0;
  int spring_iters = 0;
  bool converged = true;
  double first_force = 0.0;      // largest spring force of the first step / (k dbar_spr)
  std::vector<int32_t> nbr;      // [n][6], -1 pads pentagons
  std::vector<uint8_t> deg;      // 5 or 6
  std::vector<Vec3> pos;         // cell points (unit sphere)
  std::vector<double> area;      // control-volume area (unit sphere)
  std::vector<double> div_coef;  // [n][7][3]
  std::vector<double> lap_coef;  // [n][6]
  std::vector<int32_t> dd_idx;   // [n][18] two-ring columns, -1 pad
  std::vector<double> dd_w;      // [n][18][3] lap(grad .) weights
};

int build_grid(const thor_grid_params &p, Grid &G);

void set_error(const std::string &msg);
void clear_error();

}  // namespace thor

struct thor_mlp;
namespace thor {
// Input width, output width and largest batch of a corrector network.
void mlp_shape_of(const thor_mlp *m, int *in, int *out, int *max_batch);

}  // namespace thor

struct thor_grid {
  thor::Grid g;
};
