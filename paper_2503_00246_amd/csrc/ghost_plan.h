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

// Box scatter: the cells are cut into bricks of B^d cells.  A workgroup handles one brick: it applies
// every face with a cell in the brick (a face whose two cells lie in different bricks is visited by
// both, each expanding only into its own cell; the shared node plane goes to the lower cell's brick),
// sums the contributions over the brick's node box [org, org + kB] in a dense LDS accumulator and
// writes its nodes straight to y, except nodes on box faces that an earlier box (in box order) also
// touches: those go into halo slots, which a second kernel adds into y.
struct Box {
  int32_t org[3];         // node origin k*B*b (0 for unused axes)
  int32_t visit_first, visit_count;
  int32_t run_first, run_count;   // inspection runs (BoxRun)
  int32_t line_first, line_count; // device form: touched x-lines of the box (BoxLine)
  int32_t halo_first;             // first halo slot of the box (its slots are consecutive)
};

// One touched x-line of a box node box: bit x of `touched` marks box node x of the line as a node the
// box contributes to; bit x of `shared` marks it as a node an earlier box (in box order) already writes
// to y (this box's value goes to halo slot slot_base + (number of shared bits below x) instead).
struct BoxLine {
  uint64_t touched, shared;
  int32_t line;        // ry + E * rz (box-relative line coordinates, E = box_extent)
  int32_t slot_base;
};

// Packed face visit: c0 | c1 << 20 | c2 << 40 | axis << 60 | half << 62, half 0 = whole patch,
// 1 = lower cell (patch planes 0..k), 2 = upper cell (planes k+1..2k).  A face's primary visit (the one
// that counts it in reductions) is the one with half 0 or 1.
using Visit = uint64_t;

// A chunk of the interior Laplacian: `count` consecutive inside cells of one x-row, the first with
// lattice index `base` of its first node.
struct CellChunk {
  int64_t base;
  int32_t count, pad;
};

struct BoxRun {          // a run of touched box nodes along x
  int64_t start;         // lattice index of the first node
  int32_t acc;           // box-linear index x + E*(y + E*z) of the first node (E = box_extent)
  int32_t len;
  int32_t slot;          // -1: exclusive, written to y; else first halo slot of the run
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

  // box layout
  int brick = 0;                       // cells per brick edge
  int box_nodes = 0;                   // k*brick + 1
  std::vector<Box> boxes;              // launch order
  std::vector<Visit> visits;
  std::vector<BoxRun> box_runs;       // inspection form of the flush
  std::vector<BoxLine> box_lines;      // device form
  int64_t n_visits = 0;
  int64_t n_slots = 0;                 // halo slots
  std::vector<int64_t> halo_node;      // support nodes with halo slots (lattice index): the n_halo_single
                                       // nodes with one slot, then the others, each group ascending
  int64_t n_halo_single = 0;
  std::vector<int32_t> halo_ptr;       // slots of halo_node[h]: halo_slot[halo_ptr[h] .. halo_ptr[h+1])
  std::vector<int32_t> halo_slot;

  std::vector<Run> support_runs;       // union of face patches
  int64_t n_support = 0;
  std::vector<Run> active_runs;        // nodes of active cells
  int64_t n_active = 0;

  // inside cells (the interior Laplacian): each run of consecutive inside cells along x cut into chunks
  // of at most cell_chunk(dim, k+1) cells, grouped by colour (chunk index in the run mod 2) +
  // 2 (c1 mod 2) + 4 (c2 mod 2), so that no two chunks of a colour share a node
  std::vector<CellChunk> inside_chunks;
  int64_t n_inside = 0;  // distinct nodes of the inside cells
  int64_t inside_colour_begin[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

  // 1D tables, rounded from long double
  std::vector<double> jumps;   // k x (2k+1)
  std::vector<double> mass;    // (k+1) x (k+1)
  std::vector<double> nodes;   // k+1 GLL nodes on [0,1]
  std::vector<double> weights; // k+1 GLL weights on [0,1]
  std::vector<double> mix;     // k x k order coupling of the macro-patch form
};

// Builds the plan; returns an empty string on success or an error message.
std::string build_plan(Plan &p, int dim, const int n[3], const double lo[3], double h, int k,
                       int ls_kind, const double centre[3], double radius,
                       const signed char *cell_class, int n_balls, const double *balls, bool coloured);

// Box layout (see Box).  Called by build_plan.
std::string build_box_layout(Plan &p);

// Reference 1D stiffness on [0, 1], A[a][b] = integral of l_a' l_b' ((k+1)-point Gauss, exact), made
// exactly symmetric and centro-symmetric; for the interior-cell Laplacian.
void stiffness_1d(int k, std::vector<long double> &stiff);

// Order coupling of the macro-patch stabilisation (§2.2, its alternative form), k x k, orders i, j =
// 1..k: H[i][j] = integral over [-1, 1] of t^(i+j) dt / (i! j!), zero for i + j odd.  On the
// reference patch (two unit cells, face at t = 0) the difference of the two cells' polynomial
// extensions has degree k and vanishes at the face, and its Taylor coefficients about the face are
// the derivative jumps g_j . u over j! (up to one sign, which cancels in products).  So the patch
// integral of the product of two such differences is sum_ij (g_i . u) H[i][j] (g_j . v): the rank-k
// penalty with a k x k coupling of the orders in place of a diagonal.
void macro_mix_1d(int k, std::vector<long double> &mix);

// 1D tables in extended precision (exposed for the host tests through the ABI).
void tables_1d(int k, std::vector<long double> &nodes, std::vector<long double> &weights,
               std::vector<long double> &jumps, std::vector<long double> &mass);

}  // namespace ghost
