// Compile-time shape of the face kernel, shared by the host plan (batching) and the kernels.
#pragma once

namespace ghost {

constexpr int kMaxDegree = 7;
constexpr int kBlockThreads = 256;

// Box scatter: cells per brick edge, chosen so that a brick's node box (k*B + 1 nodes per axis) fits
// the accumulator extent E (16 in 3D, 64 in 2D).  The accumulator is E^d values; node (x, y, z) of the
// box lives at slot box_slot(x, y, z): each x-line is rotated by (5y + 11z) mod E, which spreads the
// lanes of a face (consecutive y or z) over the LDS banks for every face orientation.
#ifndef GHOST_BOX_SPAN
#define GHOST_BOX_SPAN 15
#endif
constexpr int box_extent(int dim) { return dim == 3 ? 16 : 64; }
constexpr int box_cells(int dim, int k) {
  return dim == 3 ? (GHOST_BOX_SPAN / k > 0 ? GHOST_BOX_SPAN / k : 1) : (box_extent(2) - 1) / k;
}
constexpr int box_nodes(int dim, int k) { return k * box_cells(dim, k) + 1; }
constexpr int box_acc(int dim) { return dim == 3 ? 16 * 16 * 16 : 64 * 64; }
constexpr int box_slot(int dim, int x, int y, int z) {
  return dim == 3 ? ((x + 5 * y + 11 * z) & 15) + 16 * y + 256 * z : ((x + 5 * y) & 63) + 64 * y;
}

// Threads per face: one per tangential node line, (k+1)^(d-1).
constexpr int lines_per_face(int dim, int k) { return dim == 3 ? (k + 1) * (k + 1) : (k + 1); }

// Faces handled by one workgroup of kBlockThreads threads.
constexpr int faces_per_block(int dim, int k) { return kBlockThreads / lines_per_face(dim, k); }

}  // namespace ghost
