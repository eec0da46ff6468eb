// Compile-time shape of the face kernel, shared by the host plan (batching) and the kernels.
#pragma once

namespace ghost {

constexpr int kMaxDegree = 7;
constexpr int kBlockThreads = 256;

// Box scatter: cells per brick edge, chosen so that a brick's node box (k*B + 1 nodes per axis) is
// about 16 (3D) or 64 (2D) nodes, and the padded LDS accumulator of the box.
#ifndef GHOST_BOX_SPAN
#define GHOST_BOX_SPAN 15
#endif
constexpr int box_cells(int dim, int k) { return dim == 3 ? (GHOST_BOX_SPAN / k > 0 ? GHOST_BOX_SPAN / k : 1) : 63 / k; }
constexpr int box_nodes(int dim, int k) { return k * box_cells(dim, k) + 1; }
constexpr int box_pitch(int dim, int k) { return box_nodes(dim, k) | 1; }  // odd x-pitch: fewer bank conflicts
constexpr int box_acc(int dim, int k) {
  return dim == 3 ? box_pitch(dim, k) * box_nodes(dim, k) * box_nodes(dim, k) : box_pitch(dim, k) * box_nodes(dim, k);
}

// Threads per face: one per tangential node line, (k+1)^(d-1).
constexpr int lines_per_face(int dim, int k) { return dim == 3 ? (k + 1) * (k + 1) : (k + 1); }

// Faces handled by one workgroup of kBlockThreads threads.
constexpr int faces_per_block(int dim, int k) { return kBlockThreads / lines_per_face(dim, k); }

}  // namespace ghost
