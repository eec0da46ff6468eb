// Compile-time shape of the face kernel, shared by the host plan (batching) and the kernels.
#pragma once

namespace ghost {

constexpr int kMaxDegree = 7;
constexpr int kBlockThreads = 256;

// Owner-computes accumulator capacity (entries) of one workgroup's node box.
constexpr int kDefaultAccCap = 3072;

// Threads per face: one per tangential node line, (k+1)^(d-1).
constexpr int lines_per_face(int dim, int k) { return dim == 3 ? (k + 1) * (k + 1) : (k + 1); }

// Faces handled by one workgroup of kBlockThreads threads.
constexpr int faces_per_block(int dim, int k) { return kBlockThreads / lines_per_face(dim, k); }

}  // namespace ghost
