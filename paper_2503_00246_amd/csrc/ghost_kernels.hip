// HIP kernels of the ghost-penalty operator for gfx950 (MI355X).
//
// Face kernel (Algorithm 1, face loop; §2.5.1 three-step apply in rank-k form).
// For a face with normal n and reference tables g_j (jump vectors of the two-cell patch),
// M (exact mass) and gs_j = gamma_j h^{d-1-2j} g_j, the local operator of §2.4
//     G_F = sum_j gamma_j h^{d-1-2j} (g_j g_j^T along n) (x) M (x) M
// is applied to the patch values u_F as
//     a_j = (g_j^T along n) u_F          k x (k+1)^{d-1}   normal contraction
//     b_j = (M (x) M) a_j                                  tangential masses
//     y_F = sum_j gs_j (x) b_j           (2k+1) x (k+1)^{d-1}
// which costs 2k(2k+1)(k+1)^{d-1} + 2(d-1)k(k+1)^d flops instead of the dense
// (2k+1)^2 (k+1)^{2(d-1)} of the patch matrix.
//
// Work mapping: one thread per tangential node line of a face ((k+1)^{d-1} threads per
// face), several faces of one normal axis per 256-thread workgroup.  A thread gathers its
// line of 2k+1 values along the normal straight into registers, contracts it against
// the k jump vectors, and exchanges the k values through LDS for the tangential mass
// contractions (each done by one thread per k x (k+1) line, so a line is read once).
// The expansion is again per thread and line, followed by the scatter: FP64/FP32
// hardware atomics (one launch for all faces) or plain read-modify-write within a
// race-free colour class (one launch per colour).
//
// Tables are read with wave-uniform constant indices from a read-only buffer (scalar
// loads).  Workgroup -> batch mapping is XCD-aware: the locality-ordered batch list
// is cut into 8 contiguous slices, one per XCD, so each XCD's L2 serves the overlap
// between neighbouring patches.
#include <hip/hip_runtime.h>

#include "ghost_device.h"

namespace ghost {
namespace {

constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_remap(int b, int G) {
  // Workgroups are dispatched round-robin over the XCDs: block b runs on XCD b % 8.
  const int per = G / kXcds, rem = G % kXcds;
  const int x = b % kXcds, i = b / kXcds;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// x: vector the operator acts on.  VJP: u2 is paired with the order-wise reduction
// dgamma_j += <(g_j^T) u2_F, (M (x) M)(g_j^T) x_F> over the block's faces.
template <typename T, int D, int K, bool ATOMIC, bool VJP>
__global__ __launch_bounds__(kBlockThreads) void face_kernel(
    const T *__restrict__ x, const T *__restrict__ u2, T *__restrict__ y, double *__restrict__ partial,
    const int64_t *__restrict__ face_base, const Batch *__restrict__ batches, int batch0,
    const T *__restrict__ tab, int s0, int s1, int s2) {
  constexpr int k = K - 1, NN = 2 * k + 1;
  constexpr int TL = lines_per_face(D, k), FPB = faces_per_block(D, k), NT = TL * FPB;
  __shared__ T sa[FPB * k * TL];
  __shared__ T sb[FPB * k * TL];
  const T *g = tab;
  const T *gs = tab + k * NN;
  const T *M = tab + 2 * k * NN;

  const int bl = batch0 + xcd_remap(blockIdx.x, gridDim.x);
  const Batch bt = batches[bl];
  const int tid = threadIdx.x;
  const int f = tid / TL, t = tid - f * TL;
  const bool in_block = tid < NT;
  const bool live = in_block && f < bt.count;

  int sn, st1, st2 = 0;
  if (D == 3) {
    sn = bt.axis == 0 ? s0 : (bt.axis == 1 ? s1 : s2);
    st1 = bt.axis == 0 ? s1 : s0;
    st2 = bt.axis == 2 ? s1 : s2;
  } else {
    sn = bt.axis == 0 ? s0 : s1;
    st1 = bt.axis == 0 ? s1 : s0;
  }
  const int t1 = (D == 3) ? t % K : t;
  const int t2 = (D == 3) ? t / K : 0;
  const int64_t base = live ? face_base[bt.first + f] + (int64_t)(t1 * st1 + t2 * st2) : 0;

  // ---- gather one normal line and contract it with the jump vectors
  T a[k], au[k];
#pragma unroll
  for (int j = 0; j < k; ++j) a[j] = au[j] = T(0);
  if (live) {
    T line[NN];
#pragma unroll
    for (int i = 0; i < NN; ++i) line[i] = x[base + i * sn];
#pragma unroll
    for (int j = 0; j < k; ++j) {
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < NN; ++i) acc = fma(g[j * NN + i], line[i], acc);
      a[j] = acc;
    }
    if (VJP) {
#pragma unroll
      for (int i = 0; i < NN; ++i) line[i] = u2[base + i * sn];
#pragma unroll
      for (int j = 0; j < k; ++j) {
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < NN; ++i) acc = fma(g[j * NN + i], line[i], acc);
        au[j] = acc;
      }
    }
  }

  // ---- tangential mass contractions through LDS
  if (in_block) {
#pragma unroll
    for (int j = 0; j < k; ++j) sa[(f * k + j) * TL + t] = a[j];
  }
  __syncthreads();
  const T *res;
  if (D == 3) {
    // along tangential axis 1: thread (t1, t2) owns line (j = t1, t2) if t1 < k
    if (in_block && t1 < k) {
      const T *row = &sa[(f * k + t1) * TL + t2 * K];
      T r[K];
#pragma unroll
      for (int m = 0; m < K; ++m) r[m] = row[m];
      T *out = &sb[(f * k + t1) * TL + t2 * K];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < K; ++m) acc = fma(M[q * K + m], r[m], acc);
        out[q] = acc;
      }
    }
    __syncthreads();
    // along tangential axis 2: thread (t1, t2) owns line (j = t2, t1) if t2 < k
    if (in_block && t2 < k) {
      const T *col = &sb[(f * k + t2) * TL + t1];
      T r[K];
#pragma unroll
      for (int m = 0; m < K; ++m) r[m] = col[m * K];
      T *out = &sa[(f * k + t2) * TL + t1];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < K; ++m) acc = fma(M[q * K + m], r[m], acc);
        out[q * K] = acc;
      }
    }
    __syncthreads();
    res = sa;
  } else {
    if (in_block && t < k) {
      const T *row = &sa[(f * k + t) * TL];
      T r[K];
#pragma unroll
      for (int m = 0; m < K; ++m) r[m] = row[m];
      T *out = &sb[(f * k + t) * TL];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < K; ++m) acc = fma(M[q * K + m], r[m], acc);
        out[q] = acc;
      }
    }
    __syncthreads();
    res = sb;
  }

  // ---- expand along the normal and scatter
  T c[k];
#pragma unroll
  for (int j = 0; j < k; ++j) c[j] = in_block ? res[(f * k + j) * TL + t] : T(0);
  if (live) {
#pragma unroll
    for (int i = 0; i < NN; ++i) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < k; ++j) acc = fma(gs[j * NN + i], c[j], acc);
      T *p = y + base + i * sn;
      if (ATOMIC)
        atomic_add(p, acc);
      else
        *p += acc;
    }
  }

  if (VJP) {
    // per-order partial sums of <au_j, c_j> over the block, reduced in a fixed order
    __shared__ double red[kBlockThreads / 64][k];
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int j = 0; j < k; ++j) {
      double v = live ? (double)au[j] * (double)c[j] : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    if (tid < k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kBlockThreads / 64; ++w) s += red[w][tid];
      partial[(int64_t)bl * k + tid] = s;
    }
  }
}


// Owner-computes apply.  Workgroup = one box of lattice nodes; it runs the same per-face pipeline
// as face_kernel over every face whose patch meets the box (faces crossing the box boundary are
// recomputed by each box they touch), keeps only the contributions to nodes inside the box,
// sums them in an LDS accumulator, and finally writes each owned support node once with plain,
// coalesced stores.  No global atomics, and y needs no prior zeroing.
// VJP: x = w drives du; u2 = u gives the order-wise reduction, counted once per face (on the
// face's primary visit).
template <typename T, int D, int K, bool VJP>
__global__ __launch_bounds__(kBlockThreads) void owner_kernel(
    const T *__restrict__ x, const T *__restrict__ u2, T *__restrict__ y, double *__restrict__ partial,
    const Leaf *__restrict__ leaves, const Visit *__restrict__ visits, const FlushRec *__restrict__ flushes,
    const LineRec *__restrict__ lines, int acc_bytes, const T *__restrict__ tab, int s0, int s1, int s2,
    int accumulate) {
  constexpr int k = K - 1, NN = 2 * k + 1;
  constexpr int TL = lines_per_face(D, k), FPB = faces_per_block(D, k), NT = TL * FPB;
  __shared__ T sa[FPB * k * TL];
  __shared__ T sb[FPB * k * TL];
  extern __shared__ __align__(16) unsigned char dyn_smem[];
  T *acc = reinterpret_cast<T *>(dyn_smem);
  int *table = reinterpret_cast<int *>(dyn_smem + acc_bytes);
  const T *g = tab;
  const T *gs = tab + k * NN;
  const T *M = tab + 2 * k * NN;

  const int li = xcd_remap(blockIdx.x, gridDim.x);
  const Leaf lf = leaves[li];
  const int tid = threadIdx.x;
  for (int i = tid; i < lf.acc_size; i += kBlockThreads) acc[i] = T(0);
  for (int i = tid; i < lf.line_count; i += kBlockThreads) {
    const LineRec r = lines[lf.line_first + i];
    table[r.line] = r.base;
  }
  const int f = tid / TL, t = tid - f * TL;
  const bool in_block = tid < NT;
  const int t1 = (D == 3) ? t % K : t;
  const int t2 = (D == 3) ? t / K : 0;
  const int w1 = lf.hi[1] - lf.lo[1];
  double pj[k];
#pragma unroll
  for (int j = 0; j < k; ++j) pj[j] = 0.0;
  __syncthreads();

  for (int v0 = 0; v0 < lf.visit_count; v0 += FPB) {
    const int vi = v0 + f;
    const bool live = in_block && vi < lf.visit_count;
    const Visit vis = live ? visits[lf.visit_first + vi] : Visit(0);
    const int c0 = (int)(vis & 0xFFFFF), c1 = (int)((vis >> 20) & 0xFFFFF), c2 = (int)((vis >> 40) & 0xFFFFF);
    const int axis = (int)((vis >> 60) & 3);
    const bool prim = ((vis >> 62) & 1) != 0;
    // normal axis n and tangential axes ta < tb, resolved with selects (no indexed local arrays)
    const bool ax0 = axis == 0, ax1 = axis == 1, ax2 = axis == 2;
    const int sn = ax0 ? s0 : (ax1 ? s1 : s2);
    const int st1 = ax0 ? s1 : s0;
    const int st2 = (D == 3) ? (ax2 ? s1 : s2) : 0;
    const int64_t base = (int64_t)k * ((int64_t)c0 * s0 + (int64_t)c1 * s1 + (int64_t)c2 * s2) +
                         (int64_t)(t1 * st1 + t2 * st2);

    T a[k], au[k];
#pragma unroll
    for (int j = 0; j < k; ++j) a[j] = au[j] = T(0);
    if (live) {
      T line[NN];
#pragma unroll
      for (int i = 0; i < NN; ++i) line[i] = x[base + i * sn];
#pragma unroll
      for (int j = 0; j < k; ++j) {
        T s = T(0);
#pragma unroll
        for (int i = 0; i < NN; ++i) s = fma(g[j * NN + i], line[i], s);
        a[j] = s;
      }
      if (VJP && prim) {
#pragma unroll
        for (int i = 0; i < NN; ++i) line[i] = u2[base + i * sn];
#pragma unroll
        for (int j = 0; j < k; ++j) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < NN; ++i) s = fma(g[j * NN + i], line[i], s);
          au[j] = s;
        }
      }
    }
    if (in_block) {
#pragma unroll
      for (int j = 0; j < k; ++j) sa[(f * k + j) * TL + t] = a[j];
    }
    __syncthreads();
    const T *res;
    if (D == 3) {
      if (in_block && t1 < k) {
        const T *row = &sa[(f * k + t1) * TL + t2 * K];
        T r[K];
#pragma unroll
        for (int m = 0; m < K; ++m) r[m] = row[m];
        T *out = &sb[(f * k + t1) * TL + t2 * K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
          T s = T(0);
#pragma unroll
          for (int m = 0; m < K; ++m) s = fma(M[q * K + m], r[m], s);
          out[q] = s;
        }
      }
      __syncthreads();
      if (in_block && t2 < k) {
        const T *col = &sb[(f * k + t2) * TL + t1];
        T r[K];
#pragma unroll
        for (int m = 0; m < K; ++m) r[m] = col[m * K];
        T *out = &sa[(f * k + t2) * TL + t1];
#pragma unroll
        for (int q = 0; q < K; ++q) {
          T s = T(0);
#pragma unroll
          for (int m = 0; m < K; ++m) s = fma(M[q * K + m], r[m], s);
          out[q * K] = s;
        }
      }
      __syncthreads();
      res = sa;
    } else {
      if (in_block && t < k) {
        const T *row = &sa[(f * k + t) * TL];
        T r[K];
#pragma unroll
        for (int m = 0; m < K; ++m) r[m] = row[m];
        T *out = &sb[(f * k + t) * TL];
#pragma unroll
        for (int q = 0; q < K; ++q) {
          T s = T(0);
#pragma unroll
          for (int m = 0; m < K; ++m) s = fma(M[q * K + m], r[m], s);
          out[q] = s;
        }
      }
      __syncthreads();
      res = sb;
    }
    T cj[k];
#pragma unroll
    for (int j = 0; j < k; ++j) cj[j] = in_block ? res[(f * k + j) * TL + t] : T(0);
    if (live) {
      // node coordinates: along the normal n0 + i, along the tangential axes ia, ib (fixed per thread)
      const int n0 = k * (ax0 ? c0 : (ax1 ? c1 : c2));
      const int ia = k * (ax0 ? c1 : c0) + t1;
      const int ib = (D == 3) ? k * (ax2 ? c1 : c2) + t2 : 0;
      const int lo_n = ax0 ? lf.lo[0] : (ax1 ? lf.lo[1] : lf.lo[2]);
      const int hi_n = ax0 ? lf.hi[0] : (ax1 ? lf.hi[1] : lf.hi[2]);
      const int lo_a = ax0 ? lf.lo[1] : lf.lo[0], hi_a = ax0 ? lf.hi[1] : lf.hi[0];
      const int lo_b = ax2 ? lf.lo[1] : lf.lo[2], hi_b = ax2 ? lf.hi[1] : lf.hi[2];
      bool own_t = ia >= lo_a && ia < hi_a;
      if (D == 3) own_t = own_t && ib >= lo_b && ib < hi_b;
      if (own_t) {
#pragma unroll
        for (int i = 0; i < NN; ++i) {
          const int in = n0 + i;
          if (in >= lo_n && in < hi_n) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < k; ++j) s = fma(gs[j * NN + i], cj[j], s);
            const int x0 = ax0 ? in : ia;
            const int x1 = ax1 ? in : (ax0 ? ia : ib);
            const int x2 = (D == 3) ? (ax2 ? in : ib) : 0;
            const int ln = (x1 - lf.lo[1]) + w1 * (x2 - lf.lo[2]);
            __hip_atomic_fetch_add(&acc[table[ln] + x0], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
      if (VJP && prim) {
#pragma unroll
        for (int j = 0; j < k; ++j) pj[j] += (double)au[j] * (double)cj[j];
      }
    }
    __syncthreads();  // sa / sb are reused by the next batch
  }

  // flush: 8 lanes per run of owned support nodes
  const int sub = tid >> 3, sl = tid & 7;
  for (int r = sub; r < lf.flush_count; r += kBlockThreads / 8) {
    const FlushRec fr = flushes[lf.flush_first + r];
    for (int i = sl; i < fr.len; i += 8) {
      const T v = acc[fr.acc + i];
      T *p = y + fr.start + i;
      *p = accumulate ? *p + v : v;
    }
  }

  if (VJP) {
    __shared__ double red[kBlockThreads / 64][k];
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int j = 0; j < k; ++j) {
      double v = pj[j];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    if (tid < k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kBlockThreads / 64; ++w) s += red[w][tid];
      partial[(int64_t)li * k + tid] = s;
    }
  }
}

template <typename T>
__global__ void zero_runs_kernel(T *__restrict__ y, const Run *__restrict__ runs, int n_runs) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (wave >= n_runs) return;
  const Run r = runs[wave];
  for (int i = lane; i < r.len; i += 64) y[r.start + i] = T(0);
}

// dgamma_j = hscale_j * sum_b partial[b][j], one block per order, fixed summation order.
__global__ void vjp_reduce_kernel(const double *__restrict__ partial, int n_batches, int k,
                                  const double *__restrict__ hscale, double *__restrict__ dgamma) {
  __shared__ double red[kBlockThreads];
  const int j = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int b = tid; b < n_batches; b += kBlockThreads) s += partial[(int64_t)b * k + j];
  red[tid] = s;
  __syncthreads();
  for (int w = kBlockThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) dgamma[j] = hscale[j] * red[0];
}

// gs_j = gamma_j * hscale_j * g_j in FP64, and its FP32 rounding.
__global__ void set_gamma_kernel(const double *__restrict__ gamma, int k, double *__restrict__ tab64,
                                 float *__restrict__ tab32) {
  const int NN = 2 * k + 1;
  const double *hscale = tab64 + 2 * k * NN + (k + 1) * (k + 1);
  for (int idx = threadIdx.x; idx < k * NN; idx += blockDim.x) {
    const int j = idx / NN;
    const double v = (gamma[j] * hscale[j]) * tab64[idx];
    tab64[k * NN + idx] = v;
    tab32[k * NN + idx] = (float)v;
  }
}

__global__ void fill_kernel(double *__restrict__ y, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

// Lumped GLL mass: M_ii = sum over active cells K containing node i of h^d prod_a w[i_a].
__global__ void mass_diag_kernel(double *__restrict__ diag, const Run *__restrict__ runs, int n_runs,
                                 const int8_t *__restrict__ cls, int dim, int k, int n0, int n1, int n2,
                                 int64_t L0, int64_t L1, double hd, const double *__restrict__ w) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (wave >= n_runs) return;
  const Run r = runs[wave];
  const int nn[3] = {n0, n1, n2};
  for (int i = lane; i < r.len; i += 64) {
    const int64_t idx = r.start + i;
    int64_t I[3] = {idx % L0, (idx / L0) % L1, idx / (L0 * L1)};
    int cand_c[3][2], cand_i[3][2], nc[3];
    for (int a = 0; a < 3; ++a) {
      nc[a] = 0;
      if (a >= dim) {
        cand_c[a][0] = 0;
        cand_i[a][0] = 0;
        nc[a] = 1;
        continue;
      }
      const int q = (int)(I[a] / k), rr = (int)(I[a] % k);
      if (rr == 0) {
        if (q - 1 >= 0) { cand_c[a][nc[a]] = q - 1; cand_i[a][nc[a]] = k; ++nc[a]; }
        if (q < nn[a]) { cand_c[a][nc[a]] = q; cand_i[a][nc[a]] = 0; ++nc[a]; }
      } else {
        cand_c[a][0] = q;
        cand_i[a][0] = rr;
        nc[a] = 1;
      }
    }
    double s = 0.0;
    for (int p2 = 0; p2 < nc[2]; ++p2)
      for (int p1 = 0; p1 < nc[1]; ++p1)
        for (int p0 = 0; p0 < nc[0]; ++p0) {
          const int64_t cell = cand_c[0][p0] + (int64_t)n0 * (cand_c[1][p1] + (int64_t)n1 * cand_c[2][p2]);
          if (cls[cell] == 0) continue;
          double v = w[cand_i[0][p0]] * w[cand_i[1][p1]];
          if (dim == 3) v *= w[cand_i[2][p2]];
          s += hd * v;
        }
    diag[idx] = s;
  }
}

template <typename T, bool ATOMIC, bool VJP>
hipError_t dispatch(const DevPlan &p, const T *x, const T *u2, T *y, double *partial, const T *tab,
                    int batch0, int nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const dim3 grid(nb), block(kBlockThreads);
#define GHOST_CASE(D_, K_)                                                                          \
  if (p.dim == D_ && p.k + 1 == K_) {                                                               \
    hipLaunchKernelGGL((face_kernel<T, D_, K_, ATOMIC, VJP>), grid, block, 0, s, x, u2, y, partial, \
                       p.face_base, p.batches, batch0, tab, p.stride[0], p.stride[1], p.stride[2]); \
    return hipGetLastError();                                                                       \
  }
  GHOST_CASE(2, 2) GHOST_CASE(2, 3) GHOST_CASE(2, 4) GHOST_CASE(2, 5) GHOST_CASE(2, 6) GHOST_CASE(2, 7)
  GHOST_CASE(2, 8) GHOST_CASE(3, 2) GHOST_CASE(3, 3) GHOST_CASE(3, 4) GHOST_CASE(3, 5) GHOST_CASE(3, 6)
  GHOST_CASE(3, 7) GHOST_CASE(3, 8)
#undef GHOST_CASE
  return hipErrorInvalidValue;
}


template <typename T, bool VJP>
hipError_t dispatch_owner(const DevPlan &p, const T *x, const T *u2, T *y, const T *tab, bool accumulate,
                          hipStream_t s) {
  if (p.n_leaves <= 0) return hipSuccess;
  const int acc_bytes = ((p.max_acc * (int)sizeof(T)) + 15) / 16 * 16;
  const size_t shmem = (size_t)acc_bytes + (size_t)p.max_lines * sizeof(int);
  const dim3 grid(p.n_leaves), block(kBlockThreads);
#define GHOST_OCASE(D_, K_)                                                                                     \
  if (p.dim == D_ && p.k + 1 == K_) {                                                                          \
    hipLaunchKernelGGL((owner_kernel<T, D_, K_, VJP>), grid, block, shmem, s, x, u2, y, p.vjp_partial, p.leaves, \
                       p.visits, p.flushes, p.lines, acc_bytes, tab, p.stride[0], p.stride[1], p.stride[2],   \
                       (int)accumulate);                                                                        \
    return hipGetLastError();                                                                                   \
  }
  GHOST_OCASE(2, 2) GHOST_OCASE(2, 3) GHOST_OCASE(2, 4) GHOST_OCASE(2, 5) GHOST_OCASE(2, 6) GHOST_OCASE(2, 7)
  GHOST_OCASE(2, 8) GHOST_OCASE(3, 2) GHOST_OCASE(3, 3) GHOST_OCASE(3, 4) GHOST_OCASE(3, 5) GHOST_OCASE(3, 6)
  GHOST_OCASE(3, 7) GHOST_OCASE(3, 8)
#undef GHOST_OCASE
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t zero_support(const DevPlan &p, T *y, hipStream_t s) {
  if (p.n_support_runs == 0) return hipSuccess;
  const int waves_per_block = kBlockThreads / 64;
  const int grid = (p.n_support_runs + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL((zero_runs_kernel<T>), dim3(grid), dim3(kBlockThreads), 0, s, y, p.support_runs,
                     p.n_support_runs);
  return hipGetLastError();
}

template <typename T, bool VJP>
hipError_t run_faces(const DevPlan &p, const T *x, const T *u2, T *y, const T *tab, hipStream_t s) {
  if (p.scatter == Scatter::Atomic) return dispatch<T, true, VJP>(p, x, u2, y, p.vjp_partial, tab, 0, p.n_batches, s);
  for (int c = 0; c < p.n_colours; ++c) {
    hipError_t e = dispatch<T, false, VJP>(p, x, u2, y, p.vjp_partial, tab, p.colour_begin[c],
                                           p.colour_begin[c + 1] - p.colour_begin[c], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_apply_f64(const DevPlan &p, const double *u, double *y, bool accumulate, hipStream_t s) {
  if (p.scatter == Scatter::Owner) return dispatch_owner<double, false>(p, u, nullptr, y, p.tab64, accumulate, s);
  if (!accumulate) {
    hipError_t e = zero_support(p, y, s);
    if (e != hipSuccess) return e;
  }
  return run_faces<double, false>(p, u, nullptr, y, p.tab64, s);
}

hipError_t launch_apply_f32(const DevPlan &p, const float *u, float *y, bool accumulate, hipStream_t s) {
  if (p.scatter == Scatter::Owner) return dispatch_owner<float, false>(p, u, nullptr, y, p.tab32, accumulate, s);
  if (!accumulate) {
    hipError_t e = zero_support(p, y, s);
    if (e != hipSuccess) return e;
  }
  return run_faces<float, false>(p, u, nullptr, y, p.tab32, s);
}

hipError_t launch_vjp(const DevPlan &p, const double *u, const double *w, double *du, double *dgamma,
                      bool accumulate, hipStream_t s) {
  const bool owner = p.scatter == Scatter::Owner;
  const int n_parts = owner ? p.n_leaves : p.n_batches;
  hipError_t e = hipSuccess;
  if (owner) {
    e = dispatch_owner<double, true>(p, w, u, du, p.tab64, accumulate, s);
  } else {
    if (!accumulate) e = zero_support(p, du, s);
    if (e == hipSuccess) e = run_faces<double, true>(p, w, u, du, p.tab64, s);
  }
  if (e != hipSuccess) return e;
  if (n_parts == 0) {
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, dgamma, (int64_t)p.k, 0.0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(vjp_reduce_kernel, dim3(p.k), dim3(kBlockThreads), 0, s, p.vjp_partial, n_parts,
                     p.k, p.tab64 + tab_hscale(p.k), dgamma);
  return hipGetLastError();
}

hipError_t launch_set_gamma(const DevPlan &p, const double *gamma_dev, hipStream_t s) {
  hipLaunchKernelGGL(set_gamma_kernel, dim3(1), dim3(128), 0, s, gamma_dev, p.k, p.tab64, p.tab32);
  return hipGetLastError();
}

hipError_t launch_mass_diag(const DevPlan &p, double *diag, hipStream_t s) {
  const int64_t n = p.L[0] * p.L[1] * p.L[2];
  hipLaunchKernelGGL(fill_kernel, dim3(2048), dim3(kBlockThreads), 0, s, diag, n, 0.0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.n_active_runs == 0) return e;
  double hd = p.h * p.h;
  if (p.dim == 3) hd *= p.h;
  const int waves_per_block = kBlockThreads / 64;
  const int grid = (p.n_active_runs + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(mass_diag_kernel, dim3(grid), dim3(kBlockThreads), 0, s, diag, p.active_runs,
                     p.n_active_runs, p.cls, p.dim, p.k, p.n[0], p.n[1], p.n[2], p.L[0], p.L[1], hd,
                     p.tab64 + tab_gllw(p.k));
  return hipGetLastError();
}

}  // namespace ghost
