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
// The macro-patch stabilisation (§2.2, its alternative form) runs the same steps with the orders coupled
// before the expansion, y_F = gamma_M h^{d-2} sum_i g_i (x) (sum_j H_ij b_j), H a fixed k x k matrix
// (box kernel only).
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

#include <type_traits>

#include "ghost_device.h"
#include "ghost_tables_gen.h"

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




// Per-thread view of one face visit in a box.
struct VisitPrep {
  uint32_t gofs;   // offset (elements) of the thread's normal line, patch plane 0, from the gather base
  uint32_t sn;     // lattice stride along the normal (0 for dead lanes: they read the gather base)
  int acc0, dacc;  // accumulator index of the line at patch plane 0, index stride along the normal
  bool lo, hi;     // expand patch planes 0..k / k+1..2k
  bool live, prim;
};

// glo: offset of the gather base from the box origin (<= 0), so that every gathered offset is >= 0.
template <int D, int K>
__device__ __forceinline__ VisitPrep prep_visit(Visit vis, bool live, int t1, int t2, int s1, int s2, int o0,
                                                int o1, int o2, int glo) {
  constexpr int k = K - 1, E = box_extent(D), P = box_pitch(D);
  VisitPrep q;
  const int c0 = (int)(vis & 0xFFFFF), c1 = (int)((vis >> 20) & 0xFFFFF), c2 = (int)((vis >> 40) & 0xFFFFF);
  const int axis = (int)((vis >> 60) & 3), half = (int)((vis >> 62) & 3);
  // box coordinates of the line at patch plane 0: lower cell's first node plus the tangential offsets
  // (tangential axes in increasing order: t1 along the first, t2 along the second)
  int bx = k * c0 - o0, by = k * c1 - o1, bz = (D == 3) ? k * c2 - o2 : 0;
  if (D == 3) {
    bx += axis != 0 ? t1 : 0;
    by += axis == 0 ? t1 : (axis == 2 ? t2 : 0);
    bz += axis != 2 ? t2 : 0;
  } else {
    bx += axis == 1 ? t1 : 0;
    by += axis == 0 ? t1 : 0;
  }
  q.live = live;
  q.prim = half != 2;
  q.gofs = live ? (uint32_t)(bx + s1 * by + s2 * bz - glo) : 0u;
  q.sn = live ? (uint32_t)(axis == 0 ? 1 : (axis == 1 ? s1 : s2)) : 0u;
  q.acc0 = bx + P * (by + E * bz);
  q.dacc = axis == 0 ? 1 : (axis == 1 ? P : P * E);
  q.lo = half != 2;
  q.hi = half != 1;
  return q;
}

// The 2k+1 patch values of a normal line.  A line along x (stride 1) is read in 16-byte pieces:
// a wave of x-normal faces then touches each cache line of its rows once per piece instead of once
// per value.  (The pieces are only 8-byte aligned; gfx9 global loads accept that.)
template <typename T, int NN>
__device__ __forceinline__ void gather_line(const T *__restrict__ base, uint32_t gofs, uint32_t sn, T (&out)[NN]) {
  if (sn == 1) {
    constexpr int W = 16 / (int)sizeof(T);
    typedef T V __attribute__((ext_vector_type(W), aligned(sizeof(T))));
    const V *p = reinterpret_cast<const V *>(base + gofs);
#pragma unroll
    for (int q = 0; q < NN / W; ++q) {
      const V v = p[q];
#pragma unroll
      for (int e = 0; e < W; ++e) out[q * W + e] = v[e];
    }
#pragma unroll
    for (int i = (NN / W) * W; i < NN; ++i) out[i] = base[gofs + i];
  } else {
#pragma unroll
    for (int i = 0; i < NN; ++i) out[i] = base[gofs + i * sn];
  }
}

template <int D>
using LineMask = typename std::conditional<D == 3, uint32_t, uint64_t>::type;
__device__ __forceinline__ int popc_mask(uint32_t m) { return __popc(m); }
__device__ __forceinline__ int popc_mask(uint64_t m) { return __popcll(m); }

// Dynamic box scheduling.  The blocks of a launch form up to kSchedGroups groups (blockIdx mod the
// group count: the XCD a block runs on when workgroups are dispatched round-robin over the XCDs);
// group x takes the boxes of one contiguous range of the brick order, one ticket at a time from its
// counter.  A block stops after its first ticket past the range; the last block of a group to do so
// resets the group's counters, so every launch starts from zero.
// An LDS address as the LDS address space pointer the copy builtin takes.
__device__ __forceinline__ __attribute__((address_space(3))) void *lds_ptr(char *p) {
  return (__attribute__((address_space(3))) void *)p;
}

// s_waitcnt immediate: vector-memory count 0, the other counters left at their maximum.
constexpr int kWaitVmcnt0 = (7 << 4) | (15 << 8);

// A ticket is drawn in two steps so that the atomic's latency overlaps work: draw_ticket issues it,
// settle_ticket (called once its result is needed) maps it to a box or to -1 past the range.
__device__ __forceinline__ int draw_ticket(BoxSched *s, int grp) { return atomicAdd(&s->ctr[grp], 1); }
__device__ __forceinline__ int settle_ticket(BoxSched *s, int grp, int t, int lo, int hi, int nblk) {
  if (lo + t < hi) return lo + t;
  if (atomicAdd(&s->done[grp], 1) == nblk - 1) {
    atomicExch(&s->ctr[grp], 0);
    atomicExch(&s->done[grp], 0);
  }
  return -1;
}
__device__ __forceinline__ int take_box(BoxSched *s, int grp, int lo, int hi, int nblk) {
  return settle_ticket(s, grp, draw_ticket(s, grp), lo, hi, nblk);
}

// Lattice index of a box's origin, and the offset (<= 0) from it of the gather base: the lowest node a
// visit of the box can read is one cell below the box along some axis; gathers use 32-bit offsets
// from that base.
__device__ __forceinline__ int gather_low(int o0, int o1, int o2, int k, int s1, int s2, int64_t &base) {
  base = (int64_t)o0 + (int64_t)s1 * o1 + (int64_t)s2 * o2;
  const int64_t reach = (int64_t)k * (1 + s1 + s2);
  return -(int)(base < reach ? base : reach);
}

// A visit record of the current box, read from LDS.  The next box's records may be on their way into
// the other half of the same array by LDS DMA, and the compiler, unable to tell the two halves apart,
// would make this read wait for every global load the wave has in flight (the next gather among them).
// The read is written out with its own wait instead; its address never meets the DMA's.
__device__ __forceinline__ Visit read_visit(const Visit *p) {
  Visit v;
  const uint32_t a = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const Visit *)p;
  asm volatile("ds_read_b64 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(a) : "memory");
  return v;
}

// Accumulator add in LDS, without return.  Written out for the same reason as read_visit: the compiler
// cannot tell the accumulator from the destination of the records' LDS DMA either.  (LDS operations of
// one wave complete in order, and every barrier waits for all of them.)
__device__ __forceinline__ void acc_add(double *p, double v) {
  const uint32_t a = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) double *)p;
  asm volatile("ds_add_f64 %0, %1" : : "v"(a), "v"(v) : "memory");
}

// Box fields as wave-uniform scalars.
struct BoxScalars {
  int o0, o1, o2, visit_first, visit_count, line_first, line_count, halo_first;
};
__device__ __forceinline__ BoxScalars load_box(const Box *__restrict__ boxes, int b) {
  const Box *bp = boxes + __builtin_amdgcn_readfirstlane(b);
  BoxScalars r;
  r.o0 = __builtin_amdgcn_readfirstlane(bp->org[0]);
  r.o1 = __builtin_amdgcn_readfirstlane(bp->org[1]);
  r.o2 = __builtin_amdgcn_readfirstlane(bp->org[2]);
  r.visit_first = __builtin_amdgcn_readfirstlane(bp->visit_first);
  r.visit_count = __builtin_amdgcn_readfirstlane(bp->visit_count);
  r.line_first = __builtin_amdgcn_readfirstlane(bp->line_first);
  r.line_count = __builtin_amdgcn_readfirstlane(bp->line_count);
  r.halo_first = __builtin_amdgcn_readfirstlane(bp->halo_first);
  return r;
}

// Orders a wave's LDS writes before its later reads by other lanes of the same wave (LDS executes a
// wave's instructions in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads also waits for every global load and
// store the wave has in flight; the box kernel's waves never read each other's global stores, and its
// gathers are meant to stay in flight across the barriers between boxes.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Copy a box's visits and line records from global memory into LDS in 16-byte pieces, one per lane,
// without holding them in registers (waves past the last piece issue nothing).  Addresses are a uniform
// base plus a 32-bit lane offset (the record arrays are far below 4 GB), so no 64-bit per-lane pointer
// stays live across the box.
template <int kLinesMax>
__device__ __forceinline__ void copy_box_records(const Visit *__restrict__ visits, const BoxLine *__restrict__ lines,
                                                 const BoxScalars &bn, Visit *svis_dst, BoxLine *slines_dst, int tid) {
  constexpr int kVisitPieces = kMaxBoxVisits * (int)sizeof(Visit) / 16;
  constexpr int kLinePieces = kLinesMax * (int)sizeof(BoxLine) / 16;
  const int vp = (bn.visit_count * (int)sizeof(Visit) + 15) / 16;
  const int lp = (bn.line_count * (int)sizeof(BoxLine) + 15) / 16;
  const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);  // wave-uniform: the LDS base goes to M0
  const uint32_t lane_ofs = 16u * (uint32_t)tid;
  if (wbase < kVisitPieces && tid < vp)
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const char *>(visits) +
                                         ((uint32_t)bn.visit_first * (uint32_t)sizeof(Visit) + lane_ofs),
                                     lds_ptr(reinterpret_cast<char *>(svis_dst) + 16 * wbase), 16, 0, 0);
  if (wbase < kLinePieces && tid < lp)
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const char *>(lines) +
                                         ((uint32_t)bn.line_first * (uint32_t)sizeof(BoxLine) + lane_ofs),
                                     lds_ptr(reinterpret_cast<char *>(slines_dst) + 16 * wbase), 16, 0, 0);
}

// The per-face rank-k pipeline, one wave slot (a face's tangential lines) at a time; the box kernel and
// the single-face microbenchmark share it.  Tab1d<K> holds the reference jump vectors g and mass M.
template <typename T, int K, bool VJP>
__device__ __forceinline__ void face_contract(const T (&line)[2 * K - 1], const T (&uline)[2 * K - 1], T (&a)[K - 1],
                                              T (&au)[K - 1]) {
  constexpr int k = K - 1, NN = 2 * k + 1;
  using Tab = gen::Tab1d<K>;
  // normal contraction a_j = g_j . line, folded with the reflection symmetry g_j[2k-i] = (-1)^(j+1)
  // g_j[i] (derivative order j+1 odd for even j here: those rows use the sums, the others the
  // differences); rows of dead faces are computed on node-0 data and never expanded
  {
    T ev[k], od[k], eu[k], ou[k];
#pragma unroll
    for (int i = 0; i < k; ++i) {
      ev[i] = line[i] + line[2 * k - i];
      od[i] = line[i] - line[2 * k - i];
      if (VJP) {
        eu[i] = uline[i] + uline[2 * k - i];
        ou[i] = uline[i] - uline[2 * k - i];
      }
    }
#pragma unroll
    for (int j = 0; j < k; ++j) {
      T s, su = T(0);
      if (j % 2 == 0) {
        s = T(Tab::g[j * NN + k]) * line[k];
        if (VJP) su = T(Tab::g[j * NN + k]) * uline[k];
#pragma unroll
        for (int i = 0; i < k; ++i) {
          s = fma(T(Tab::g[j * NN + i]), ev[i], s);
          if (VJP) su = fma(T(Tab::g[j * NN + i]), eu[i], su);
        }
      } else {
        s = T(0);
#pragma unroll
        for (int i = 0; i < k; ++i) {
          s = fma(T(Tab::g[j * NN + i]), od[i], s);
          if (VJP) su = fma(T(Tab::g[j * NN + i]), ou[i], su);
        }
      }
      a[j] = s;
      au[j] = su;
    }
  }
}

template <typename T, int D, int K>
__device__ __forceinline__ void face_masses(T *sa, int f, int t, int t1, int t2, bool in_block) {
  constexpr int k = K - 1, TL = lines_per_face(D, k);
  using Tab = gen::Tab1d<K>;
  // tangential masses in place: each row (column) is read and rewritten by the one thread that owns
  // it, and the wavefront fence between the passes orders the row writes before the column reads
  if (D == 3) {
    if (in_block && t1 < k) {
      T *row = &sa[(f * k + t1) * TL + t2 * K];
      T r[K];
#pragma unroll
      for (int m = 0; m < K; ++m) r[m] = row[m];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        T s = T(0);
#pragma unroll
        for (int m = 0; m < K; ++m) s = fma(T(Tab::M[q * K + m]), r[m], s);
        row[q] = s;
      }
    }
    wave_sync();
    if (in_block && t2 < k) {
      T *col = &sa[(f * k + t2) * TL + t1];
      T r[K];
#pragma unroll
      for (int m = 0; m < K; ++m) r[m] = col[m * K];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        T s = T(0);
#pragma unroll
        for (int m = 0; m < K; ++m) s = fma(T(Tab::M[q * K + m]), r[m], s);
        col[q * K] = s;
      }
    }
    wave_sync();
  } else {
    if (in_block && t < k) {
      T *row = &sa[(f * k + t) * TL];
      T r[K];
#pragma unroll
      for (int m = 0; m < K; ++m) r[m] = row[m];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        T s = T(0);
#pragma unroll
        for (int m = 0; m < K; ++m) s = fma(T(Tab::M[q * K + m]), r[m], s);
        row[q] = s;
      }
    }
    wave_sync();
  }
}

// Order coupling of the macro-patch form: m_i = sum_j H[i][j] c_j, H zero for i + j odd.
template <typename T, int K>
__device__ __forceinline__ void macro_mix(const T (&cj)[K - 1], T (&m)[K - 1]) {
  constexpr int k = K - 1;
  using Tab = gen::Tab1d<K>;
#pragma unroll
  for (int i = 0; i < k; ++i) {
    T s = T(0);
#pragma unroll
    for (int j = i % 2; j < k; j += 2) s = fma(T(Tab::H[i * k + j]), cj[j], s);
    m[i] = s;
  }
}

// Expansion onto the patch line from the scaled order values cs_j (derivative form: coef_j c_j with
// coef_j = gamma_j h^{d-1-2j}; macro-patch form: gamma_M h^{d-2} m_j).
template <typename T, int K>
__device__ __forceinline__ void face_expand(const T (&cs)[K - 1], T (&yv2)[2 * K - 1]) {
  constexpr int k = K - 1, NN = 2 * k + 1;
  using Tab = gen::Tab1d<K>;
  // y_i = sum_j g_j[i] cs_j, folded: E_i from the symmetric orders, O_i from the others,
  // y_i = E_i + O_i and y_{2k-i} = E_i - O_i
#pragma unroll
  for (int i = 0; i <= k; ++i) {
    T e = T(0), o = T(0);
#pragma unroll
    for (int j = 0; j < k; ++j) {
      if (j % 2 == 0)
        e = fma(T(Tab::g[j * NN + i]), cs[j], e);
      else if (i < k)
        o = fma(T(Tab::g[j * NN + i]), cs[j], o);
    }
    yv2[i] = e + o;
    if (i < k) yv2[2 * k - i] = e - o;
  }
}

// Flush plan of a box, one packed word per flush line of the lane: -1 when the lane's node is not
// touched, else the box line index (bits 0-7), a shared flag (bit 8) and, for a shared node, its halo
// slot relative to the box's first (bits 9-21).  All records are read before any is decoded, and the
// decode has no branches.
template <int D, int kLines, int kGroups>
__device__ __forceinline__ void decode_lines(const BoxLine *slines, int grp, LineMask<D> gbit, int line_count,
                                             int halo_first, int (&fl)[kLines]) {
  using Mask = LineMask<D>;
  BoxLine bl[kLines];
#pragma unroll
  for (int m = 0; m < kLines; ++m) bl[m] = slines[grp + m * kGroups];
#pragma unroll
  for (int m = 0; m < kLines; ++m) {
    const Mask tm = (Mask)bl[m].touched, sm = (Mask)bl[m].shared;
    const bool touched = grp + m * kGroups < line_count && (tm & gbit) != 0;
    const bool sh = (sm & gbit) != 0;
    const int rel = bl[m].slot_base - halo_first + popc_mask(sm & (gbit - 1));
    fl[m] = touched ? (bl[m].line | (sh ? (1 << 8) | (rel << 9) : 0)) : -1;
  }
}

// Box apply (default scatter).  A box is (part of) one brick of cells: the kernel runs the per-face
// pipeline of face_kernel over the box's face visits, expanding only into the brick's cells (a face
// split between two bricks is visited twice, once per half), and sums the results in a dense LDS
// accumulator over the brick's node box (odd row pitch, so the lanes of a face spread over the banks).
// Every node is then written to y with a plain store by the first box (in box order) that touches it;
// later boxes touching it store their part into halo slots, which halo_kernel adds into y.  No global
// atomics on y, and y needs no prior zeroing.
// A face's tangential lines never straddle a wavefront (64 / (k+1)^(d-1) faces per wave), so the
// mass passes exchange values through the wave's own LDS rows without workgroup barriers: each wave
// works through its faces of the box independently, and the workgroup meets once per box.
// The workgroups are persistent: each takes boxes from the scheduler and, while it works on one box,
// already loads the next box's visits and line records; the gather of the next box's first faces is
// issued before the flush of this one.
// VJP: x = w drives du; u2 = u gives the order-wise reduction, counted on each face's primary visit,
// and stored per box so that the reduction order does not depend on the schedule.
// MACRO: the macro-patch stabilisation, whose orders are coupled by H before the expansion (and whose
// one coefficient's reduction pairs u's orders with the coupled w values).
template <typename T, int D, int K, bool VJP, bool MACRO>
__device__ __forceinline__ void box_body(
    const T *__restrict__ x, const T *__restrict__ u2, T *__restrict__ y, T *__restrict__ halo,
    double *__restrict__ partial, const Box *__restrict__ boxes, const Visit *__restrict__ visits,
    const BoxLine *__restrict__ lines, const T *__restrict__ tab, int s1, int s2, int accumulate, int n_boxes,
    BoxSched *__restrict__ sched) {
  constexpr int k = K - 1, NN = 2 * k + 1;
  // faces never straddle a wavefront: FW faces per wave, FPB per round over the workgroup
  constexpr int TL = lines_per_face(D, k), FW = 64 / TL, FPB = box_faces_per_batch(D, k);
  static_assert(TL <= 64, "a face must fit one wavefront");
  constexpr int E = box_extent(D), P = box_pitch(D), ACC = box_acc(D);
  constexpr int kLinesMax = D == 3 ? E * E : E;
  // jump vectors and mass matrix as compile-time constants (folded into the instructions); only the
  // gamma-dependent factors coef_j = gamma_j h^{d-1-2j} come from the table buffer
  using Tab = gen::Tab1d<K>;
  T coef[k];
#pragma unroll
  for (int j = 0; j < k; ++j) coef[j] = tab[tab_coef(k) + j];
  // The accumulator is FP64 in both precisions: LDS adds of doubles are served at a far higher rate
  // than adds of floats on this hardware, and the FP32 path gains the exact summation of its
  // contributions.
  using A = double;
  __shared__ A acc[ACC];
  __shared__ T sa[FPB * k * TL];  // per-face k x (k+1)^(d-1) values, transformed in place
  __shared__ Visit svis[2][kMaxBoxVisits];  // visits of the current box and of the next one
  __shared__ BoxLine slines[kLinesMax];     // line records of the current box, then of the next one
  __shared__ int s_box[2];
  const int tid = threadIdx.x;

  // scheduling group and its box range
  const int nblocks = gridDim.x, ng = min(kSchedGroups, nblocks), sg = blockIdx.x % ng;
  const int nblk = nblocks / ng + (sg < nblocks % ng ? 1 : 0);
  const int lo = (int)((int64_t)n_boxes * sg / ng), hi = (int)((int64_t)n_boxes * (sg + 1) / ng);

  // per-thread constants: face slot and tangential line of the face pipeline, flush lane group
  const int lane_w = tid & 63, fw = lane_w / TL;
  const int f = (tid >> 6) * FW + fw, t = lane_w - fw * TL;
  const bool in_block = fw < FW;
  const int t1 = (D == 3) ? t % K : t;
  const int t2 = (D == 3) ? t / K : 0;
  // Flush plan: a group of E lanes takes touched x-lines grp, grp + kGroups, ... of the box, lane = box
  // x coordinate, so the stores of a group are consecutive; kLines lines per group cover the box.
  constexpr int kGroups = kBoxThreads / E, kLines = kLinesMax / kGroups;
  static_assert(kGroups * kLines == kLinesMax, "flush groups must cover the box lines");
  const int grp = tid / E, gx = tid % E;
  using Mask = LineMask<D>;
  const Mask gbit = (Mask)1 << gx;

  // first two boxes of this workgroup
  if (tid == 0) {
    const int b0 = take_box(sched, sg, lo, hi, nblk);
    s_box[0] = b0;
    s_box[1] = b0 >= 0 ? take_box(sched, sg, lo, hi, nblk) : -1;
  }
  __syncthreads();
  int cur = __builtin_amdgcn_readfirstlane(s_box[0]);
  int nxt = __builtin_amdgcn_readfirstlane(s_box[1]);
  if (cur < 0) return;
  BoxScalars bc = load_box(boxes, cur);
  if (tid < bc.visit_count) svis[0][tid] = visits[bc.visit_first + tid];
  if (tid < bc.line_count) slines[tid] = lines[bc.line_first + tid];
  __syncthreads();
  int64_t box_base;
  int glo = gather_low(bc.o0, bc.o1, bc.o2, k, s1, s2, box_base);
  VisitPrep nxp = prep_visit<D, K>(in_block && f < bc.visit_count ? svis[0][f] : Visit(0),
                                   in_block && f < bc.visit_count, t1, t2, s1, s2, bc.o0, bc.o1, bc.o2, glo);
  T lnext[NN], unext[NN];
  gather_line<T, NN>(x + (box_base + glo), nxp.gofs, nxp.sn, lnext);
  if (VJP) gather_line<T, NN>(u2 + (box_base + glo), nxp.gofs, nxp.sn, unext);
  int buf = 0;
  int fl[kLines];
  decode_lines<D, kLines, kGroups>(slines, grp, gbit, bc.line_count, bc.halo_first, fl);
  // The accumulator is zeroed once here; afterwards each box's flush clears the nodes it read, which
  // are exactly the nodes its visits added into, so every box starts from zero.
#pragma unroll
  for (int i = 0; i < (ACC + kBoxThreads - 1) / kBoxThreads; ++i)
    if (i * kBoxThreads + tid < ACC) acc[i * kBoxThreads + tid] = A(0);
  // acc zeroed and the first box's line records decoded before any wave adds into acc or copies the
  // next box's records over them
  lds_barrier();

  for (;;) {
    // ---- box `cur`: its visits are in svis[buf], its line records in slines, and the gather of its
    // first round is in flight in lnext / unext
    T *const yb = y + box_base;
    BoxScalars bn{};
    int64_t nbase = 0;
    int nglo = 0;
    if (nxt >= 0) {
      bn = load_box(boxes, nxt);
      nglo = gather_low(bn.o0, bn.o1, bn.o2, k, s1, s2, nbase);
    }
    int ticket = 0;  // draws the box after `nxt` (thread 0); settled at the end of this box
    if (tid == 0 && nxt >= 0) ticket = draw_ticket(sched, sg);
    // (the flush plan fl of this box was decoded before the barrier that ended the previous box, which
    // also ordered the previous flush's clearing of acc before this box's adds)
    double pj[k];
#pragma unroll
    for (int j = 0; j < k; ++j) pj[j] = 0.0;
    // Copy the next box's visits and line records straight from global memory into LDS (16 bytes per
    // lane, no registers held); each wave waits for its copies before the barrier that ends the box.
    // A wave issues them in its first round, behind the gather of its second (so that no wait for a
    // gather also waits for them), or here when it has at most one round.  The global arrays are
    // padded so that the last 16-byte piece stays inside them.
    // Each wave works through its own faces of the box (round b: visit b * FPB + f) and stops after
    // its last; no workgroup barrier is needed until the box is done.  (The round count is
    // wave-uniform, made visible as such to the compiler so that the round's branches are scalar.)
    const int wave_first = __builtin_amdgcn_readfirstlane((tid >> 6) * FW);
    const int nbat = bc.visit_count > wave_first ? (bc.visit_count - wave_first + FPB - 1) / FPB : 0;
    if (nxt >= 0 && nbat <= 1)
      copy_box_records<kLinesMax>(visits, lines, bn, &svis[buf ^ 1][0], slines, tid);
    T yv[kLines];
    for (int b = 0; b < nbat; ++b) {
      const VisitPrep cur_p = nxp;
      const bool last = b + 1 == nbat;
      // the next round's visit record, read before this round's contraction waits for its gather
      const int vi = (b + 1) * FPB + f;
      const bool vlive = !last && in_block && vi < bc.visit_count;
      const Visit vrec = vlive ? read_visit(&svis[buf][vi]) : Visit(0);
      T line[NN], uline[NN];
#pragma unroll
      for (int i = 0; i < NN; ++i) {
        line[i] = lnext[i];
        uline[i] = VJP ? unext[i] : T(0);
      }

      T a[k], au[k];
      face_contract<T, K, VJP>(line, uline, a, au);
      if (in_block) {
#pragma unroll
        for (int j = 0; j < k; ++j) sa[(f * k + j) * TL + t] = a[j];
      }
      wave_sync();
      if (last && accumulate) {  // y at the exclusive flush nodes
#pragma unroll
        for (int m = 0; m < kLines; ++m) {
          const unsigned line = (unsigned)fl[m] & 0xFF;
          const bool excl = fl[m] >= 0 && !(fl[m] & (1 << 8));
          yv[m] = yb[excl ? (uint32_t)(gx + s1 * (int)(line % E) + s2 * (int)(line / E)) : 0u];
        }
      }
      // issue the next gather: the next round of this box (the next box's first round is gathered after
      // the barrier that ends this box)
      if (!last) {
        nxp = prep_visit<D, K>(vrec, vlive, t1, t2, s1, s2, bc.o0, bc.o1, bc.o2, glo);
        gather_line<T, NN>(x + (box_base + glo), nxp.gofs, nxp.sn, lnext);
        if (VJP) gather_line<T, NN>(u2 + (box_base + glo), nxp.gofs, nxp.sn, unext);
        if (b == 0 && nxt >= 0) copy_box_records<kLinesMax>(visits, lines, bn, &svis[buf ^ 1][0], slines, tid);
      }
      face_masses<T, D, K>(sa, f, t, t1, t2, in_block);
      T cj[k];
#pragma unroll
      for (int j = 0; j < k; ++j) cj[j] = in_block ? sa[(f * k + j) * TL + t] : T(0);
      if (cur_p.live) {
        T cs[k];
        if (MACRO) {
          T hm[k];
          macro_mix<T, K>(cj, hm);
#pragma unroll
          for (int j = 0; j < k; ++j) cs[j] = coef[0] * hm[j];
          if (VJP && cur_p.prim) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < k; ++j) s += (double)au[j] * (double)hm[j];
            pj[0] += s;
          }
        } else {
#pragma unroll
          for (int j = 0; j < k; ++j) cs[j] = coef[j] * cj[j];
          if (VJP && cur_p.prim) {
#pragma unroll
            for (int j = 0; j < k; ++j) pj[j] += (double)au[j] * (double)cj[j];
          }
        }
        T yv2[NN];
        face_expand<T, K>(cs, yv2);
        if (cur_p.lo) {
          int off = cur_p.acc0;
#pragma unroll
          for (int i = 0; i <= k; ++i, off += cur_p.dacc)
            acc_add(&acc[off], (A)yv2[i]);
        }
        if (cur_p.hi) {
          int off = cur_p.acc0 + (k + 1) * cur_p.dacc;
#pragma unroll
          for (int i = k + 1; i < NN; ++i, off += cur_p.dacc)
            acc_add(&acc[off], (A)yv2[i]);
        }
      }
      wave_sync();  // sa is reused by this wave's next round
    }
    if (nbat == 0 && accumulate) {  // a wave without faces in this box still flushes its lines
#pragma unroll
      for (int m = 0; m < kLines; ++m) {
        const unsigned line = (unsigned)fl[m] & 0xFF;
        const bool excl = fl[m] >= 0 && !(fl[m] & (1 << 8));
        yv[m] = yb[excl ? (uint32_t)(gx + s1 * (int)(line % E) + s2 * (int)(line / E)) : 0u];
      }
    }
    // all waves done with this box: acc complete; the next box's records (copied by every wave, each
    // waiting for its own copies) visible; then its first gather overlaps the flush.  The ticket drawn
    // at the top of the box has returned too: thread 0 publishes the box after `nxt` now, so that no
    // wave waits for its flush stores at the barrier that ends the box.
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    lds_barrier();
    if (tid == 0) s_box[0] = nxt >= 0 ? settle_ticket(sched, sg, ticket, lo, hi, nblk) : -1;
    if (nxt >= 0) {
      const bool live = in_block && f < bn.visit_count;
      const Visit v = live ? svis[buf ^ 1][f] : Visit(0);
      nxp = prep_visit<D, K>(v, live, t1, t2, s1, s2, bn.o0, bn.o1, bn.o2, nglo);
      gather_line<T, NN>(x + (nbase + nglo), nxp.gofs, nxp.sn, lnext);
      if (VJP) gather_line<T, NN>(u2 + (nbase + nglo), nxp.gofs, nxp.sn, unext);
    }

    // flush: exclusive nodes to y, shared ones to their halo slot.  Every lane first reads and clears its
    // accumulator slots (a lane without a node on a line uses the pad column of row 0, which no face adds
    // into), so that the reads are issued together; then the stores follow.
    int ai[kLines];
    A av[kLines];
#pragma unroll
    for (int m = 0; m < kLines; ++m) ai[m] = fl[m] >= 0 ? gx + P * (int)((unsigned)fl[m] & 0xFF) : E;
#pragma unroll
    for (int m = 0; m < kLines; ++m) av[m] = acc[ai[m]];
#pragma unroll
    for (int m = 0; m < kLines; ++m) acc[ai[m]] = A(0);
#pragma unroll
    for (int m = 0; m < kLines; ++m) {
      if (fl[m] >= 0) {
        const unsigned line = (unsigned)fl[m] & 0xFF;
        A v = av[m];
        if (fl[m] & (1 << 8)) {
          halo[bc.halo_first + (fl[m] >> 9)] = (T)v;
        } else {
          if (accumulate) v += (A)yv[m];
          yb[(uint32_t)(gx + s1 * (int)(line % E) + s2 * (int)(line / E))] = (T)v;
        }
      }
    }
    if (VJP) {
      __shared__ double red[kBoxThreads / 64][k];
      const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
      for (int j = 0; j < k; ++j) {
        double v = pj[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[wave][j] = v;
      }
      lds_barrier();
      if (tid < k) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < kBoxThreads / 64; ++w) sum += red[w][tid];
        partial[(int64_t)cur * k + tid] = sum;
      }
    }
    // the next box's flush plan, from its line records (in LDS since the barrier that ended this box)
    if (nxt >= 0) decode_lines<D, kLines, kGroups>(slines, grp, gbit, bn.line_count, bn.halo_first, fl);
    // acc read and cleared by the flush before the next box adds into it; slines decoded before the
    // next box's copies refill it; s_box published
    lds_barrier();
    if (nxt < 0) break;
    cur = nxt;
    bc = bn;
    box_base = nbase;
    glo = nglo;
    nxt = __builtin_amdgcn_readfirstlane(s_box[0]);
    buf ^= 1;
  }
}

#define GHOST_BOX_PARAMS                                                                                  \
  const T *__restrict__ x, const T *__restrict__ u2, T *__restrict__ y, T *__restrict__ halo,             \
      double *__restrict__ partial, const Box *__restrict__ boxes, const Visit *__restrict__ visits,      \
      const BoxLine *__restrict__ lines, const T *__restrict__ tab, int s1, int s2, int accumulate,     \
      int n_boxes, BoxSched *__restrict__ sched
#define GHOST_BOX_ARGS x, u2, y, halo, partial, boxes, visits, lines, tab, s1, s2, accumulate, n_boxes, sched

// Two blocks of 512 threads per CU need at most 128 VGPRs (4 waves per SIMD); the compiler is held to
// that for the apply (FP32 at every degree and FP64 up to k = 4 fit without spilling; FP64 at k = 5 and
// 6 spills a few values, reloaded once per box; at k = 6 one of them is also stored once per face round).
// The VJP and the FP64 apply at k = 7 carry more live values and run one block per CU instead: spilled
// values reloaded behind a gather would make the flush wait for it.
template <typename T, int D, int K, bool VJP, bool MACRO>
__global__ __launch_bounds__(kBoxThreads) __attribute__((amdgpu_waves_per_eu(4))) void box_kernel(
    GHOST_BOX_PARAMS) {
  box_body<T, D, K, VJP, MACRO>(GHOST_BOX_ARGS);
}

template <typename T, int D, int K, bool VJP, bool MACRO>
__global__ __launch_bounds__(kBoxThreads) void box_kernel_wide(GHOST_BOX_PARAMS) {
  box_body<T, D, K, VJP, MACRO>(GHOST_BOX_ARGS);
}
#undef GHOST_BOX_PARAMS
#undef GHOST_BOX_ARGS

// y[node] += sum of the node's halo slots, for every node more than one box touches (the first box to
// touch it has already written y there, in either mode).  The first n_single nodes have one slot, at
// slot[h]: their loads do not wait on a pointer.
template <typename T>
__global__ void halo_kernel(T *__restrict__ y, const T *__restrict__ halo, const int64_t *__restrict__ node,
                            const int32_t *__restrict__ ptr, const int32_t *__restrict__ slot, int n,
                            int n_single) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= n) return;
  T *p = y + node[h];
  T s;
  if (h < n_single) {
    s = halo[slot[h]];
  } else {
    s = T(0);
    for (int q = ptr[h]; q < ptr[h + 1]; ++q) s += halo[slot[q]];
  }
  *p += s;
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

// gs_j = gamma_j * hscale_j * g_j and coef_j = gamma_j * hscale_j in FP64, and their FP32 roundings,
// for the ng coefficients of the context (k, or 1 for the macro-patch form).
__device__ void write_gamma_tables(const double *gamma, int ng, int k, double *__restrict__ tab64,
                                   float *__restrict__ tab32) {
  const int NN = 2 * k + 1;
  const double *hscale = tab64 + tab_hscale(k);
  for (int idx = threadIdx.x; idx < ng * NN; idx += blockDim.x) {
    const int j = idx / NN;
    const double v = (gamma[j] * hscale[j]) * tab64[idx];
    tab64[k * NN + idx] = v;
    tab32[k * NN + idx] = (float)v;
  }
  for (int j = threadIdx.x; j < ng; j += blockDim.x) {
    const double c = gamma[j] * hscale[j];
    tab64[tab_coef(k) + j] = c;
    tab32[tab_coef(k) + j] = (float)c;
  }
}

__global__ void set_gamma_kernel(const double *__restrict__ gamma, int ng, int k, double *__restrict__ tab64,
                                 float *__restrict__ tab32) {
  write_gamma_tables(gamma, ng, k, tab64, tab32);
}

// Same, with gamma passed by value from the host.
__global__ void set_gamma_host_kernel(GammaArg g, int ng, int k, double *__restrict__ tab64,
                                      float *__restrict__ tab32) {
  write_gamma_tables(g.v, ng, k, tab64, tab32);
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


template <typename T, int D, int K, bool VJP, bool MACRO>
void launch_box(const DevPlan &p, const T *x, const T *u2, T *y, T *halo, const T *tab, bool accumulate,
                hipStream_t s) {
  // persistent workgroups: as many as fit on the device at once (the first launch asks the runtime)
  const void *fn;
  // the VJP and the FP64 apply at k = 7 hold too many live values for 128 VGPRs: one block per CU
  constexpr bool kWide = VJP || (sizeof(T) == 8 && K == 8);
  if constexpr (kWide)
    fn = reinterpret_cast<const void *>(&box_kernel_wide<T, D, K, VJP, MACRO>);
  else
    fn = reinterpret_cast<const void *>(&box_kernel<T, D, K, VJP, MACRO>);
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBoxThreads, 0) != hipSuccess || nb < 1) nb = 1;
    per_cu = nb;
  }
  const int resident = per_cu * (p.n_cu > 0 ? p.n_cu : 1);
  const dim3 grid(p.n_boxes < resident ? p.n_boxes : resident), block(kBoxThreads);
  if constexpr (kWide)
    hipLaunchKernelGGL((box_kernel_wide<T, D, K, VJP, MACRO>), grid, block, 0, s, x, u2, y, halo, p.vjp_partial, p.boxes,
                       p.visits, p.box_lines, tab, p.stride[1], p.stride[2], (int)accumulate, p.n_boxes, p.sched);
  else
    hipLaunchKernelGGL((box_kernel<T, D, K, VJP, MACRO>), grid, block, 0, s, x, u2, y, halo, p.vjp_partial, p.boxes,
                       p.visits, p.box_lines, tab, p.stride[1], p.stride[2], (int)accumulate, p.n_boxes, p.sched);
}

// Optional timing events of a launch (see DevPlan::ev).
void mark(const DevPlan &p, int i, hipStream_t s) {
  if (p.ev[i]) (void)hipEventRecord(p.ev[i], s);
}

template <typename T, bool VJP>
hipError_t dispatch_box(const DevPlan &p, const T *x, const T *u2, T *y, const T *tab, bool accumulate,
                        hipStream_t s) {
  mark(p, 0, s);
  if (p.n_boxes <= 0) {
    mark(p, 1, s);
    mark(p, 2, s);
    return hipSuccess;
  }
  T *halo = reinterpret_cast<T *>(p.halo);
  hipError_t e = hipErrorInvalidValue;
#define GHOST_BCASE(D_, K_)                                           \
  if (p.dim == D_ && p.k + 1 == K_) {                                 \
    if (p.macro)                                                      \
      launch_box<T, D_, K_, VJP, true>(p, x, u2, y, halo, tab, accumulate, s); \
    else                                                              \
      launch_box<T, D_, K_, VJP, false>(p, x, u2, y, halo, tab, accumulate, s); \
    e = hipGetLastError();                                            \
  }
  GHOST_BCASE(2, 2) GHOST_BCASE(2, 3) GHOST_BCASE(2, 4) GHOST_BCASE(2, 5) GHOST_BCASE(2, 6) GHOST_BCASE(2, 7)
  GHOST_BCASE(2, 8) GHOST_BCASE(3, 2) GHOST_BCASE(3, 3) GHOST_BCASE(3, 4) GHOST_BCASE(3, 5) GHOST_BCASE(3, 6)
  GHOST_BCASE(3, 7) GHOST_BCASE(3, 8)
#undef GHOST_BCASE
  mark(p, 1, s);
  if (e != hipSuccess) return e;
  if (p.n_halo > 0) {
    hipLaunchKernelGGL((halo_kernel<T>), dim3((p.n_halo + kBlockThreads - 1) / kBlockThreads), dim3(kBlockThreads),
                       0, s, y, (const T *)halo, p.halo_node, p.halo_ptr, p.halo_slot, p.n_halo, p.n_halo_single);
    e = hipGetLastError();
  }
  mark(p, 2, s);
  return e;
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

// Face-parallel scatters: the same event marks around all face kernels (there is no halo pass).
template <typename T, bool VJP>
hipError_t run_faces_marked(const DevPlan &p, const T *x, const T *u2, T *y, const T *tab, hipStream_t s) {
  mark(p, 0, s);
  const hipError_t e = run_faces<T, VJP>(p, x, u2, y, tab, s);
  mark(p, 1, s);
  mark(p, 2, s);
  return e;
}

}  // namespace

// K consecutive values of one lattice line, moved in 16-byte pieces and a scalar tail.  The pieces are
// only element-aligned, which gfx9 global loads and stores accept.
template <typename T, int K>
__device__ __forceinline__ void load_line(const T *__restrict__ p, bool live, T (&v)[K]) {
  constexpr int W = 16 / (int)sizeof(T);
  typedef T V __attribute__((ext_vector_type(W), aligned(sizeof(T))));
  if (live) {
#pragma unroll
    for (int q = 0; q < K / W; ++q) {
      const V w = reinterpret_cast<const V *>(p)[q];
#pragma unroll
      for (int e = 0; e < W; ++e) v[q * W + e] = w[e];
    }
#pragma unroll
    for (int i = (K / W) * W; i < K; ++i) v[i] = p[i];
  } else {
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] = T(0);
  }
}

template <typename T, int K>
__device__ __forceinline__ void store_line(T *__restrict__ p, const T (&v)[K]) {
  constexpr int W = 16 / (int)sizeof(T);
  typedef T V __attribute__((ext_vector_type(W), aligned(sizeof(T))));
#pragma unroll
  for (int q = 0; q < K / W; ++q) {
    V w;
#pragma unroll
    for (int e = 0; e < W; ++e) w[e] = v[q * W + e];
    reinterpret_cast<V *>(p)[q] = w;
  }
#pragma unroll
  for (int i = (K / W) * W; i < K; ++i) p[i] = v[i];
}

// Interior-cell Laplacian (the cell term of the weak form, §2.1, on the cells the boundary does not cut,
// evaluated by sum factorisation as in §2.5 and Algorithm 1): y += sum over inside cells K of K_K u_K with
//   K_K = h^{d-2} sum_a (A on axis a, M on the others),
// A and M the reference 1D stiffness and mass matrices.  One tangential x-line of a cell per lane (the
// face kernel's lane layout with the normal along x), 64 / (k+1)^(d-1) cells per wavefront; the x factors
// act within the lane, the y and z factors by rows in the wave's LDS, as in the face's mass passes:
//   3D: P = M_y (A_x u) + A_y (M_x u), Q = M_y (M_x u), result = M_z P + A_z Q;
//   2D: result = M_y (A_x u) + A_y (M_x u).
// A workgroup takes a chunk of consecutive inside cells of one x-row: the cells at even positions of the
// chunk first, then, after a workgroup barrier, those at odd positions, so that no two cells applied at
// once share a node and the rows' cache lines are reused between the two phases.  Neighbouring chunks
// of a row (one shared node) and neighbouring rows are in different launches (colours), so y is read,
// added to and written back without atomics.
// Where (k+1)^(d-1) lines do not divide a wavefront (3D k = 4, 5, 6), the cells are packed over the whole
// workgroup instead (14 rather than 8 cells per phase at k = 5), a cell may straddle two waves, and
// the passes meet at workgroup barriers instead of wavefront fences.

template <bool kDense>
__device__ __forceinline__ void cell_sync() {
  if (kDense)
    __syncthreads();
  else
    wave_sync();
}

template <typename T, int D, int K>
__global__ __launch_bounds__(kBoxThreads) void cell_kernel(const T *__restrict__ u, T *__restrict__ y,
                                                           const CellChunk *__restrict__ chunks, int s1, int s2,
                                                           T scale) {
  constexpr int TL = cell_lines(D, K), FW = 64 / TL, CPB = cells_per_block(D, K);
  constexpr bool kDense = cell_dense(D, K);
  using Tab = gen::Tab1d<K>;
  __shared__ T sp[CPB * K * TL], sq[CPB * K * TL];  // per cell: [x][t], t = t1 + K t2
  const int tid = threadIdx.x, lane_w = tid & 63, fw = lane_w / TL;
  const int c = kDense ? tid / TL : (tid >> 6) * FW + fw;
  const int t = kDense ? tid - c * TL : lane_w - fw * TL;
  const bool in_block = kDense ? c < CPB : fw < FW;
  const int t1 = (D == 3) ? t % K : t;
  const int t2 = (D == 3) ? t / K : 0;
  const CellChunk ch = chunks[blockIdx.x];
  T *P = &sp[c * K * TL], *Q = &sq[c * K * TL];
  for (int phase = 0; phase < 2; ++phase) {
    const int pos = 2 * c + phase;  // the lane's cell in the chunk
    const bool live = in_block && pos < ch.count;
    const int64_t line0 = live ? ch.base + (int64_t)(K - 1) * pos + (int64_t)s1 * t1 + (int64_t)s2 * t2 : 0;
    // the lane's x-line in 16-byte pieces (as the gather of x-normal lines), zeros for dead lanes
    T ul[K];
    load_line<T, K>(u + line0, live, ul);
    // x factors within the lane
    T mx[K], ax[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      T m = T(0), a = T(0);
#pragma unroll
      for (int x = 0; x < K; ++x) {
        m = fma(T(Tab::M[q * K + x]), ul[x], m);
        a = fma(T(Tab::A[q * K + x]), ul[x], a);
      }
      mx[q] = m;
      ax[q] = a;
    }
    if (in_block) {
#pragma unroll
      for (int x = 0; x < K; ++x) {
        P[x * TL + t] = ax[x];
        Q[x * TL + t] = mx[x];
      }
    }
    cell_sync<kDense>();
    // y factors: the lane owns row (x = t1, z = t2) of both arrays, K values along y
    if (in_block) {
      const int row = t1 * TL + K * t2;  // element y of the row at row + y
      T pa[K], qm[K];
#pragma unroll
      for (int m = 0; m < K; ++m) {
        pa[m] = P[row + m];
        qm[m] = Q[row + m];
      }
#pragma unroll
      for (int q = 0; q < K; ++q) {
        T sP = T(0), sQ = T(0);
#pragma unroll
        for (int m = 0; m < K; ++m) {
          sP = fma(T(Tab::M[q * K + m]), pa[m], sP);
          sP = fma(T(Tab::A[q * K + m]), qm[m], sP);
          sQ = fma(T(Tab::M[q * K + m]), qm[m], sQ);
        }
        P[row + q] = sP;
        if (D == 3) Q[row + q] = sQ;
      }
    }
    cell_sync<kDense>();
    if (D == 3) {
      // z factors: the lane owns row (x = t2, y = t1), K values along z at stride K
      if (in_block) {
        const int row = t2 * TL + t1;
        T pa[K], qm[K];
#pragma unroll
        for (int m = 0; m < K; ++m) {
          pa[m] = P[row + m * K];
          qm[m] = Q[row + m * K];
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
          T sR = T(0);
#pragma unroll
          for (int m = 0; m < K; ++m) {
            sR = fma(T(Tab::M[q * K + m]), pa[m], sR);
            sR = fma(T(Tab::A[q * K + m]), qm[m], sR);
          }
          P[row + q * K] = sR;
        }
      }
      cell_sync<kDense>();
    }
    if (live) {
      T yl[K];
      load_line<T, K>(y + line0, true, yl);
#pragma unroll
      for (int x = 0; x < K; ++x) yl[x] += scale * P[x * TL + t];
      store_line<T, K>(y + line0, yl);
    }
    // the even cells' updates of y (and their reads of P, Q) complete before the odd cells start
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_cell_apply_t(const DevPlan &p, const T *u, T *y, hipStream_t s) {
  const T scale = (T)(p.dim == 3 ? p.h : 1.0);  // h^{d-2}
  hipError_t e = hipSuccess;
  for (int col = 0; col < (1 << p.dim) && e == hipSuccess; ++col) {
    const int64_t b0 = p.inside_colour_begin[col], n = p.inside_colour_begin[col + 1] - b0;  // chunks
    if (n == 0) continue;
    e = hipErrorInvalidValue;
#define GHOST_CCASE(D_, K_)                                                                               \
  if (p.dim == D_ && p.k + 1 == K_) {                                                                      \
    hipLaunchKernelGGL((cell_kernel<T, D_, K_>), dim3((unsigned)n), dim3(kBoxThreads), 0, s, u, y,        \
                       p.inside_chunks + b0, p.stride[1], p.stride[2], scale);                              \
    e = hipGetLastError();                                                                                 \
  }
    GHOST_CCASE(2, 2) GHOST_CCASE(2, 3) GHOST_CCASE(2, 4) GHOST_CCASE(2, 5) GHOST_CCASE(2, 6) GHOST_CCASE(2, 7)
    GHOST_CCASE(2, 8) GHOST_CCASE(3, 2) GHOST_CCASE(3, 3) GHOST_CCASE(3, 4) GHOST_CCASE(3, 5) GHOST_CCASE(3, 6)
    GHOST_CCASE(3, 7) GHOST_CCASE(3, 8)
#undef GHOST_CCASE
  }
  return e;
}

hipError_t launch_cell_apply(const DevPlan &p, const double *u, double *y, hipStream_t s) {
  return launch_cell_apply_t<double>(p, u, y, s);
}
hipError_t launch_cell_apply_f32(const DevPlan &p, const float *u, float *y, hipStream_t s) {
  return launch_cell_apply_t<float>(p, u, y, s);
}

// Single-face microbenchmark, compute-bound (the computational-efficiency experiment of §3, ghost
// penalty only): every wave slot applies its face's operator to the same patch values `reps` times with
// the box kernel's per-face pipeline (the values are made opaque to the compiler before each repetition,
// so that none is folded away) and writes the sum, out = reps * G_F in.  Layout per face: [normal node
// i][tangential line t], t = t1 + (k+1) t2.  No gather from the lattice and no scatter.
template <typename T, int D, int K>
__global__ __launch_bounds__(kBoxThreads) void face_micro_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                                 const T *__restrict__ tab, int64_t n_faces,
                                                                 int reps) {
  constexpr int k = K - 1, NN = 2 * k + 1;
  constexpr int TL = lines_per_face(D, k), FW = 64 / TL, FPB = box_faces_per_batch(D, k);
  __shared__ T sa[FPB * k * TL];
  const int tid = threadIdx.x, lane_w = tid & 63, fw = lane_w / TL;
  const int f = (tid >> 6) * FW + fw, t = lane_w - fw * TL;
  const bool in_block = fw < FW;
  const int t1 = (D == 3) ? t % K : t;
  const int t2 = (D == 3) ? t / K : 0;
  const int64_t face = (int64_t)blockIdx.x * FPB + f;
  const bool live = in_block && face < n_faces;
  T coef[k];
#pragma unroll
  for (int j = 0; j < k; ++j) coef[j] = tab[tab_coef(k) + j];
  T line[NN], acc[NN];
#pragma unroll
  for (int i = 0; i < NN; ++i) {
    line[i] = live ? in[(face * NN + i) * TL + t] : T(0);
    acc[i] = T(0);
  }
  for (int r = 0; r < reps; ++r) {
#pragma unroll
    for (int i = 0; i < NN; ++i) asm volatile("" : "+v"(line[i]));
    T a[k], au[k];
    face_contract<T, K, false>(line, line, a, au);
    if (in_block) {
#pragma unroll
      for (int j = 0; j < k; ++j) sa[(f * k + j) * TL + t] = a[j];
    }
    wave_sync();
    face_masses<T, D, K>(sa, f, t, t1, t2, in_block);
    T cj[k];
#pragma unroll
    for (int j = 0; j < k; ++j) cj[j] = in_block ? sa[(f * k + j) * TL + t] : T(0);
    T cs[k], yv2[NN];
#pragma unroll
    for (int j = 0; j < k; ++j) cs[j] = coef[j] * cj[j];
    face_expand<T, K>(cs, yv2);
#pragma unroll
    for (int i = 0; i < NN; ++i) acc[i] += yv2[i];
    wave_sync();  // sa is rewritten by the next repetition
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < NN; ++i) out[(face * NN + i) * TL + t] = acc[i];
  }
}

template <typename T>
hipError_t launch_face_micro_t(const DevPlan &p, const T *in, T *out, const T *tab, int64_t n_faces, int reps,
                               hipStream_t s) {
  if (n_faces == 0) return hipSuccess;
  hipError_t e = hipErrorInvalidValue;
#define GHOST_MCASE(D_, K_)                                                                               \
  if (p.dim == D_ && p.k + 1 == K_) {                                                                      \
    const int64_t fpb = box_faces_per_batch(D_, K_ - 1);                                                   \
    hipLaunchKernelGGL((face_micro_kernel<T, D_, K_>), dim3((unsigned)((n_faces + fpb - 1) / fpb)),       \
                       dim3(kBoxThreads), 0, s, in, out, tab, n_faces, reps);                              \
    e = hipGetLastError();                                                                                 \
  }
  GHOST_MCASE(2, 2) GHOST_MCASE(2, 3) GHOST_MCASE(2, 4) GHOST_MCASE(2, 5) GHOST_MCASE(2, 6) GHOST_MCASE(2, 7)
  GHOST_MCASE(2, 8) GHOST_MCASE(3, 2) GHOST_MCASE(3, 3) GHOST_MCASE(3, 4) GHOST_MCASE(3, 5) GHOST_MCASE(3, 6)
  GHOST_MCASE(3, 7) GHOST_MCASE(3, 8)
#undef GHOST_MCASE
  return e;
}

hipError_t launch_face_micro(const DevPlan &p, const double *in, double *out, int64_t n_faces, int reps,
                             hipStream_t s) {
  return launch_face_micro_t<double>(p, in, out, p.tab64, n_faces, reps, s);
}
hipError_t launch_face_micro_f32(const DevPlan &p, const float *in, float *out, int64_t n_faces, int reps,
                                 hipStream_t s) {
  return launch_face_micro_t<float>(p, in, out, p.tab32, n_faces, reps, s);
}

hipError_t launch_apply_f64(const DevPlan &p, const double *u, double *y, bool accumulate, hipStream_t s) {
  if (p.scatter == Scatter::Box) return dispatch_box<double, false>(p, u, nullptr, y, p.tab64, accumulate, s);
  if (!accumulate) {
    hipError_t e = zero_support(p, y, s);
    if (e != hipSuccess) return e;
  }
  return run_faces_marked<double, false>(p, u, nullptr, y, p.tab64, s);
}

hipError_t launch_apply_f32(const DevPlan &p, const float *u, float *y, bool accumulate, hipStream_t s) {
  if (p.scatter == Scatter::Box) return dispatch_box<float, false>(p, u, nullptr, y, p.tab32, accumulate, s);
  if (!accumulate) {
    hipError_t e = zero_support(p, y, s);
    if (e != hipSuccess) return e;
  }
  return run_faces_marked<float, false>(p, u, nullptr, y, p.tab32, s);
}

hipError_t launch_vjp(const DevPlan &p, const double *u, const double *w, double *du, double *dgamma,
                      bool accumulate, hipStream_t s) {
  const bool box = p.scatter == Scatter::Box;
  const int n_parts = box ? p.n_boxes : p.n_batches;
  hipError_t e = hipSuccess;
  if (box) {
    e = dispatch_box<double, true>(p, w, u, du, p.tab64, accumulate, s);
  } else {
    if (!accumulate) e = zero_support(p, du, s);
    if (e == hipSuccess) e = run_faces_marked<double, true>(p, w, u, du, p.tab64, s);
  }
  if (e != hipSuccess) return e;
  if (n_parts == 0) {
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, dgamma, (int64_t)p.n_gamma, 0.0);
    return hipGetLastError();
  }
  // partial holds k values per box or batch; the first n_gamma are reduced
  hipLaunchKernelGGL(vjp_reduce_kernel, dim3(p.n_gamma), dim3(kBlockThreads), 0, s, p.vjp_partial, n_parts,
                     p.k, p.tab64 + tab_hscale(p.k), dgamma);
  return hipGetLastError();
}

hipError_t launch_set_gamma(const DevPlan &p, const double *gamma_dev, hipStream_t s) {
  hipLaunchKernelGGL(set_gamma_kernel, dim3(1), dim3(128), 0, s, gamma_dev, p.n_gamma, p.k, p.tab64, p.tab32);
  return hipGetLastError();
}

hipError_t launch_set_gamma_host(const DevPlan &p, GammaArg g, hipStream_t s) {
  hipLaunchKernelGGL(set_gamma_host_kernel, dim3(1), dim3(128), 0, s, g, p.n_gamma, p.k, p.tab64, p.tab32);
  return hipGetLastError();
}

// diag[node] += the diagonal of G at every patch node of every face: for the patch node at normal
// position i and tangential positions (t1, t2), sum_j coef_j g_j[i]^2 M[t1][t1] M[t2][t2] (the
// diagonal of the Kronecker factors, §2.4); for the macro-patch form coef_0 sum_ab H[a][b] g_a[i] g_b[i]
// in place of the sum.  One workgroup per face batch; FP64 atomics (setup-time use by the
// preconditioned CG).
__global__ void ghost_diag_kernel(double *__restrict__ diag, const int64_t *__restrict__ face_base,
                                  const Batch *__restrict__ batches, const double *__restrict__ tab, int dim, int k,
                                  int macro, int s0, int s1, int s2) {
  const Batch bt = batches[blockIdx.x];
  const int K = k + 1, NN = 2 * k + 1;
  const int np = NN * K * (dim == 3 ? K : 1);
  const double *g = tab, *M = tab + tab_M(k), *coef = tab + tab_coef(k);
  const int axis = bt.axis;
  const int sn = axis == 0 ? s0 : (axis == 1 ? s1 : s2);
  const int st1 = axis == 0 ? s1 : s0;
  const int st2 = dim == 3 ? (axis == 2 ? s1 : s2) : 0;
  for (int idx = threadIdx.x; idx < bt.count * np; idx += blockDim.x) {
    const int f = idx / np, q = idx - f * np;
    const int i = q % NN, t = q / NN, t1 = t % K, t2 = t / K;
    double gi = 0.0;
    if (macro) {
      const double *H = tab + tab_mix(k);
      for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) gi += H[a * k + b] * g[a * NN + i] * g[b * NN + i];
      gi *= coef[0];
    } else {
      for (int j = 0; j < k; ++j) gi += coef[j] * g[j * NN + i] * g[j * NN + i];
    }
    const double v = gi * M[t1 * K + t1] * (dim == 3 ? M[t2 * K + t2] : 1.0);
    atomicAdd(&diag[face_base[bt.first + f] + (int64_t)i * sn + (int64_t)t1 * st1 + (int64_t)t2 * st2], v);
  }
}

hipError_t launch_zero_support(const DevPlan &p, double *y, hipStream_t s) { return zero_support(p, y, s); }

hipError_t launch_ghost_diag(const DevPlan &p, double *diag, hipStream_t s) {
  if (p.n_batches == 0) return hipSuccess;
  hipLaunchKernelGGL(ghost_diag_kernel, dim3(p.n_batches), dim3(kBlockThreads), 0, s, diag, p.face_base, p.batches,
                     (const double *)p.tab64, p.dim, p.k, (int)p.macro, p.stride[0], p.stride[1], p.stride[2]);
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
