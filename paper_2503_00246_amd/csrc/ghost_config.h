// Compile-time shape of the face kernel, shared by the host plan (batching) and the kernels.
#pragma once

namespace ghost {

constexpr int kMaxDegree = 7;
constexpr int kBlockThreads = 256;

// Box scatter: cells per brick edge, chosen so that a brick's node box (k*B + 1 nodes per axis) fits
// the accumulator extent E (16 in 3D, 64 in 2D; also the lanes of one flush group).  Node (x, y, z) of
// the box sits at accumulator index x + P*(y + E*z) with the odd row pitch P = E + 1, which spreads
// the lanes of a face (consecutive tangential nodes) over the LDS banks for every face orientation.
#ifndef GHOST_BOX_SPAN
#define GHOST_BOX_SPAN 15
#endif
constexpr int box_extent(int dim) { return dim == 3 ? 16 : 64; }
constexpr int box_pitch(int dim) { return box_extent(dim) + 1; }
constexpr int box_cells(int dim, int k) {
  return dim == 3 ? (GHOST_BOX_SPAN / k > 0 ? GHOST_BOX_SPAN / k : 1) : (box_extent(2) - 1) / k;
}
constexpr int box_nodes(int dim, int k) { return k * box_cells(dim, k) + 1; }
constexpr int box_acc(int dim) { return dim == 3 ? box_pitch(3) * 16 * 16 : box_pitch(2) * 64; }
// Box kernel workgroup size; a box holds at most one visit per thread (bricks with more visits are
// split into several boxes over the same node box).
constexpr int kBoxThreads = 512;
constexpr int kMaxBoxVisits = kBoxThreads;
// halo slots of one box, numbered from the box's first (a box touches at most its 16^3 / 64^2 nodes)
constexpr int kMaxBoxHalo = 1 << 13;

// Interior-cell Laplacian: one x-line of a cell per lane, (k+1)^(d-1) lines per cell.  Where they do not
// divide a wavefront (3D k = 4, 5, 6) the cells are packed over the whole workgroup (dense layout).
// A workgroup takes a chunk of up to 2 * cells_per_block consecutive inside cells of one x-row.
constexpr int cell_lines(int dim, int K) { return dim == 3 ? K * K : K; }
constexpr bool cell_dense(int dim, int K) {
  return kBoxThreads / cell_lines(dim, K) > (kBoxThreads / 64) * (64 / cell_lines(dim, K));
}
constexpr int cells_per_block(int dim, int K) {
  return cell_dense(dim, K) ? kBoxThreads / cell_lines(dim, K) : (kBoxThreads / 64) * (64 / cell_lines(dim, K));
}
constexpr int cell_chunk(int dim, int K) { return 2 * cells_per_block(dim, K); }

// Threads per face: one per tangential node line, (k+1)^(d-1).
constexpr int lines_per_face(int dim, int k) { return dim == 3 ? (k + 1) * (k + 1) : (k + 1); }

// Faces handled by one workgroup of kBlockThreads threads, and per batch of the box kernel.
constexpr int faces_per_block(int dim, int k) { return kBlockThreads / lines_per_face(dim, k); }
// box kernel: a face never straddles a wavefront, 64 / lines faces per wave
constexpr int box_faces_per_batch(int dim, int k) { return (kBoxThreads / 64) * (64 / lines_per_face(dim, k)); }

}  // namespace ghost
