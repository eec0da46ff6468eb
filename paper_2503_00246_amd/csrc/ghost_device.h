// Device-side view of a plan and the kernel launchers (implemented in ghost_kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "ghost_plan.h"

namespace ghost {

// Layout of the per-context table buffers (offsets in elements of the precision):
//   [0, k*NN)            g    : reference jump vectors, row j-1 = order j
//   [k*NN, 2*k*NN)       gs   : gamma_j h^{d-1-2j} g_j, the expansion coefficients of one face
//   [2*k*NN, +K*K)       M    : reference mass matrix
//   [.., +k)             coef : gamma_j h^{d-1-2j}
//   FP64 buffer only: [.., +k) hscale_j = h^{d-1-2j}, then [.., +K) GLL weights on [0, 1], then
//   [.., +k*k) the order coupling H of the macro-patch form
// Macro-patch contexts have one coefficient gamma_M: coef_0 = gamma_M h^{d-2}, hscale_0 = h^{d-2}, the
// other coef / hscale entries and the gs rows past the first are zero.
__host__ __device__ constexpr int tab_gs(int k) { return k * (2 * k + 1); }
__host__ __device__ constexpr int tab_M(int k) { return 2 * k * (2 * k + 1); }
__host__ __device__ constexpr int tab_coef(int k) { return tab_M(k) + (k + 1) * (k + 1); }
__host__ __device__ constexpr int tab_hscale(int k) { return tab_coef(k) + k; }
__host__ __device__ constexpr int tab_gllw(int k) { return tab_hscale(k) + k; }
__host__ __device__ constexpr int tab_mix(int k) { return tab_gllw(k) + k + 1; }
__host__ __device__ constexpr int tab_size64(int k) { return tab_mix(k) + k * k; }
__host__ __device__ constexpr int tab_size32(int k) { return tab_hscale(k); }

enum class Scatter { Box = 0, Atomic = 1, Coloured = 2 };

// Ticket counters of the persistent box kernel, one pair per scheduling group; zero between launches.
constexpr int kSchedGroups = 8;
struct BoxSched {
  int ctr[kSchedGroups];
  int done[kSchedGroups];
};

struct DevPlan {
  int dim = 0, k = 0;
  bool macro = false;  // macro-patch stabilisation in place of the derivative-jump penalty
  int n_gamma = 0;     // coefficients: k (derivative form) or 1 (macro-patch form)
  Scatter scatter = Scatter::Box;
  int32_t stride[3] = {1, 1, 1};
  int n[3] = {1, 1, 1};
  int64_t L[3] = {1, 1, 1};
  double h = 0;

  const int64_t *face_base = nullptr;
  const Batch *batches = nullptr;
  int n_batches = 0;
  bool coloured = false;
  int n_colours = 0;
  const int *colour_begin = nullptr;  // host array, n_colours + 1

  const Run *support_runs = nullptr;
  int n_support_runs = 0;
  const Run *active_runs = nullptr;
  int n_active_runs = 0;
  const int8_t *cls = nullptr;        // device cell classes

  // box layout (default scatter)
  const Box *boxes = nullptr;
  const Visit *visits = nullptr;
  const BoxLine *box_lines = nullptr;
  int n_boxes = 0;
  void *halo = nullptr;               // n_slots values of the apply's precision
  const int64_t *halo_node = nullptr;
  const int32_t *halo_ptr = nullptr;
  const int32_t *halo_slot = nullptr;
  int n_halo = 0;
  int n_halo_single = 0;              // halo_node[0, n_halo_single) have the one slot halo_slot[h]
  BoxSched *sched = nullptr;          // zero-initialised at setup
  int n_cu = 0;                       // compute units of the device
  // optional timing events: recorded before the scatter kernels, between them and the halo pass,
  // and after it (all null: no records)
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};

  // inside cells of the interior Laplacian (first-node lattice index), by parity colour
  const CellChunk *inside_chunks = nullptr;
  int64_t inside_colour_begin[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

  double *tab64 = nullptr;
  float *tab32 = nullptr;
  double *vjp_partial = nullptr;      // max(n_batches, n_boxes) * k doubles
};

hipError_t launch_apply_f64(const DevPlan &p, const double *u, double *y, bool accumulate, hipStream_t s);
hipError_t launch_apply_f32(const DevPlan &p, const float *u, float *y, bool accumulate, hipStream_t s);
hipError_t launch_vjp(const DevPlan &p, const double *u, const double *w, double *du, double *dgamma,
                      bool accumulate, hipStream_t s);
hipError_t launch_set_gamma(const DevPlan &p, const double *gamma_dev, hipStream_t s);
struct GammaArg {  // gamma by value, for host-side updates
  double v[kMaxDegree];
};
hipError_t launch_set_gamma_host(const DevPlan &p, GammaArg g, hipStream_t s);
hipError_t launch_mass_diag(const DevPlan &p, double *diag, hipStream_t s);
hipError_t launch_ghost_diag(const DevPlan &p, double *diag, hipStream_t s);  // diag += diag(G)
hipError_t launch_zero_support(const DevPlan &p, double *y, hipStream_t s);
// interior-cell Laplacian: y += sum over inside cells of K_K u_K (sum factorised, one launch per colour)
hipError_t launch_cell_apply(const DevPlan &p, const double *u, double *y, hipStream_t s);
hipError_t launch_cell_apply_f32(const DevPlan &p, const float *u, float *y, hipStream_t s);
// single-face microbenchmark: out = reps * G_F in per face, local layout [normal node][tangential line]
hipError_t launch_face_micro(const DevPlan &p, const double *in, double *out, int64_t n_faces, int reps,
                             hipStream_t s);
hipError_t launch_face_micro_f32(const DevPlan &p, const float *in, float *out, int64_t n_faces, int reps,
                                 hipStream_t s);

}  // namespace ghost
