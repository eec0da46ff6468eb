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

// Owner-computes scatter: a box of lattice nodes [lo, hi) owned by one workgroup, which applies every
// face whose patch meets the box, accumulates the box's share in LDS and writes each owned support
// node once.
struct Leaf {
  int32_t lo[3], hi[3];   // owned node ranges per axis
  int32_t visit_first, visit_count;
  int32_t flush_first, flush_count;
  int32_t line_first, line_count;
  int32_t acc_size;       // accumulator entries (sum of per-line spans)
  int32_t pad;
};

// Packed face visit: lower cell c0 | c1 << 20 | c2 << 40 | axis << 60 | primary << 62.  The primary visit
// of a face is the one by the box owning the face's first patch node (used to count it once).
using Visit = uint64_t;

struct FlushRec {        // a run of owned support nodes along x and its place in the accumulator
  int64_t start;         // lattice index of the first node
  int32_t len;
  int32_t acc;           // accumulator offset of the first node
};

struct LineRec {         // accumulator base of one owned x-line: acc offset of node x is base + x
  int32_t line;          // (I1 - lo1) + (hi1 - lo1) * (I2 - lo2)
  int32_t base;
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

  // owner-computes layout
  int brick = 0;                       // cells per brick edge before splitting
  std::vector<Leaf> leaves;            // launch order
  std::vector<Visit> visits;
  std::vector<FlushRec> flushes;
  std::vector<LineRec> lines;
  int64_t n_visits = 0;
  int max_acc = 0, max_lines_box = 0;  // largest accumulator and line table over the leaves

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

// Owner-computes layout for brick edge `brick` (cells) and accumulator capacity `acc_cap` (entries);
// bricks whose accumulator would exceed the capacity are split.  Called by build_plan.
std::string build_owner_layout(Plan &p, int brick, int acc_cap);

// Default brick edge for a dimension and degree.
int default_brick(int dim, int k);

// 1D tables in extended precision (exposed for the host tests through the ABI).
void tables_1d(int k, std::vector<long double> &nodes, std::vector<long double> &weights,
               std::vector<long double> &jumps, std::vector<long double> &mass);

}  // namespace ghost
