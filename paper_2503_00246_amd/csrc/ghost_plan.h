// Host-side plan of the ghost-penalty operator: everything computed once at setup.
// Pure C++17, no HIP.  Shared by the C ABI and the kernel launchers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "ghost_config.h"
#include "ghost.h"

namespace ghost {

struct Batch {          // one workgroup of the face kernel: up to faces_per_block faces, one normal axis
  int32_t first;        // index of the first face in Plan::face_base
  int16_t count;        // faces in the batch
  int8_t axis;          // normal axis
  int8_t colour;        // colour class (-1 when not coloured)
};

struct Run {            // maximal run of consecutive lattice nodes along x
  int64_t start;
  int32_t len;
  int32_t pad;
};

struct Plan {
  int dim = 0, k = 0;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0};
  double h = 0;
  int64_t L[3] = {1, 1, 1};       // lattice nodes per axis
  int64_t stride[3] = {1, 1, 1};  // linear-index stride per axis
  int64_t n_lattice = 0;

  std::vector<int8_t> cls;        // cell classes, x fastest
  int64_t n_active_cells = 0, n_cut_cells = 0;

  // faces per normal axis: lower-cell multi-index, colour
  std::vector<int32_t> face_cell[3];   // 3 ints per face
  std::vector<int8_t> face_colour[3];

  // launch order
  bool coloured = false;
  int n_colours = 0;
  std::vector<Batch> batches;
  std::vector<int64_t> face_base;      // lattice index of patch node (0,..,0), in batch order
  std::vector<int> colour_begin;       // coloured: batch range [colour_begin[c], colour_begin[c+1])

  std::vector<Run> support_runs;       // union of face patches
  int64_t n_support = 0;
  std::vector<Run> active_runs;        // nodes of active cells
  int64_t n_active = 0;

  // 1D tables, rounded from long double
  std::vector<double> jumps;   // k x (2k+1)
  std::vector<double> mass;    // (k+1) x (k+1)
  std::vector<double> nodes;   // k+1 GLL nodes on [0,1]
  std::vector<double> weights; // k+1 GLL weights on [0,1]
};

// Builds the plan; returns an empty string on success or an error message.
std::string build_plan(Plan &p, int dim, const int n[3], const double lo[3], double h, int k,
                       int ls_kind, const double centre[3], double radius,
                       const signed char *cell_class, bool coloured);

// 1D tables in extended precision (exposed for the host tests through the ABI).
void tables_1d(int k, std::vector<long double> &nodes, std::vector<long double> &weights,
               std::vector<long double> &jumps, std::vector<long double> &mass);

}  // namespace ghost
