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



constexpr int kVisitChunk = 256;
constexpr int kBoxThreads = 512;  // box kernel block size: 2 x the faces of a 256-thread batch in flight


// Per-thread view of one face visit in a box: lattice address of the thread's normal line, the normal
// stride, the line's box coordinates and the expanded plane range.
struct VisitPrep {
  int64_t base;          // lattice index of the thread's normal line, patch plane 0
  int sn;                // lattice stride along the normal
  int axis, rn, ra, rb;  // normal axis; box coordinates: normal origin, tangential a / b of the line
  int ilo, ihi;          // expanded patch planes
  bool live, prim;
};

template <int D, int K>
__device__ __forceinline__ VisitPrep prep_visit(Visit vis, bool live, int t1, int t2, int s0, int s1, int s2,
                                                int o0, int o1, int o2) {
  constexpr int k = K - 1;
  VisitPrep q;
  q.live = live;
  const int c0 = (int)(vis & 0xFFFFF), c1 = (int)((vis >> 20) & 0xFFFFF), c2 = (int)((vis >> 40) & 0xFFFFF);
  const int axis = (int)((vis >> 60) & 3);
  const int half = (int)((vis >> 62) & 3);
  q.axis = axis;
  q.prim = half != 2;
  const bool ax0 = axis == 0, ax1 = axis == 1, ax2 = axis == 2;
  // lattice strides along the normal and the tangential axes (ta < tb)
  q.sn = ax0 ? s0 : (ax1 ? s1 : s2);
  const int st1 = ax0 ? s1 : s0;
  const int st2 = (D == 3) ? (ax2 ? s1 : s2) : 0;
  q.base = (int64_t)k * ((int64_t)c0 * s0 + (int64_t)c1 * s1 + (int64_t)c2 * s2) + (int64_t)(t1 * st1 + t2 * st2);
  if (!live) {  // dead lanes load node 0 (unconditional loads keep the gather free of branches)
    q.base = 0;
    q.sn = 0;
  }
  // box-relative coordinates
  const int r0 = k * c0 - o0, r1 = k * c1 - o1, r2 = (D == 3) ? k * c2 - o2 : 0;
  q.rn = ax0 ? r0 : (ax1 ? r1 : r2);
  q.ra = (ax0 ? r1 : r0) + t1;
  q.rb = (D == 3) ? (ax2 ? r1 : r2) + t2 : 0;
  q.ilo = half == 2 ? k + 1 : 0;
  q.ihi = half == 1 ? k : 2 * k;
  return q;
}

// Box apply (default scatter).  Workgroup = one brick of cells; it runs the per-face pipeline of
// face_kernel over every face with a cell in the brick, expanding only into the brick's cells (a face
// split between two bricks is visited twice, once per half), and sums the results in a dense LDS
// accumulator over the brick's node box.  Nodes that no other box contains are then written to y
// with plain stores; nodes on shared box faces go to halo slots that halo_kernel adds into y.
// No global atomics, and y needs no prior zeroing.
// VJP: x = w drives du; u2 = u gives the order-wise reduction, counted on each face's primary visit.
template <typename T, int D, int K, bool VJP>
__device__ __forceinline__ void box_body(
    const T *__restrict__ x, const T *__restrict__ u2, T *__restrict__ y, T *__restrict__ halo,
    double *__restrict__ partial, const Box *__restrict__ boxes, const Visit *__restrict__ visits,
    const BoxLine *__restrict__ lines, const T *__restrict__ tab, int s0, int s1, int s2, int accumulate) {
  constexpr int k = K - 1, NN = 2 * k + 1;
  constexpr int TL = lines_per_face(D, k), FPB = kBoxThreads / TL, NT = TL * FPB;
  constexpr int E = box_extent(D), ACC = box_acc(D);
  __shared__ T acc[ACC];
  __shared__ T sa[FPB * k * TL];  // per-face k x (k+1)^(d-1) values, transformed in place
  const T *g = tab;
  const T *gs = tab + k * NN;
  const T *M = tab + 2 * k * NN;

  const int bi = xcd_remap(blockIdx.x, gridDim.x);
  // box fields as wave-uniform scalars (kept in SGPRs)
  const Box *bp = boxes + bi;
  const int o0 = __builtin_amdgcn_readfirstlane(bp->org[0]);
  const int o1 = __builtin_amdgcn_readfirstlane(bp->org[1]);
  const int o2 = __builtin_amdgcn_readfirstlane(bp->org[2]);
  const int visit_first = __builtin_amdgcn_readfirstlane(bp->visit_first);
  const int visit_count = __builtin_amdgcn_readfirstlane(bp->visit_count);
  const int line_first = __builtin_amdgcn_readfirstlane(bp->line_first);
  const int line_count = __builtin_amdgcn_readfirstlane(bp->line_count);
  const int tid = threadIdx.x;
  const int64_t box_base = (int64_t)o0 + (int64_t)s1 * o1 + (int64_t)s2 * o2;
  // Flush plan: a group of E lanes takes touched x-lines grp, grp + kGroups, ... of the box, lane = box
  // x coordinate, so the stores of a group are consecutive; kLines lines per group cover the box.
  constexpr int kGroups = kBoxThreads / E, kLines = ACC / (E * kGroups);
  static_assert(kGroups * kLines * E == ACC, "flush groups must cover the accumulator");
  const int grp = tid / E, gx = tid % E;
  const uint64_t gbit = (uint64_t)1 << gx;
  // Issue every global load of the prologue before waiting on any: the box's lines, its first visits.
  BoxLine bl[kLines];
  const int lc1 = max(line_count - 1, 0);
#pragma unroll
  for (int m = 0; m < kLines; ++m) bl[m] = lines[line_first + min(grp + m * kGroups, lc1)];
  const int nv0 = min(visit_count, kVisitChunk);
  const Visit v_first = visits[visit_first + min(tid, max(nv0 - 1, 0))];
  for (int i = tid; i < ACC; i += kBoxThreads) acc[i] = T(0);
  // Per line: fa = accumulator slot | shared flag << 12 (-1: the lane's node is not touched);
  // fs = y offset from the box origin (exclusive node) or halo slot (shared node).
  int fa[kLines], fs[kLines];
  T yv[kLines];
#pragma unroll
  for (int m = 0; m < kLines; ++m) {
    const bool touched = grp + m * kGroups < line_count && (bl[m].touched & gbit);
    const bool sh = (bl[m].shared & gbit) != 0;
    const int ry = bl[m].line % E, rz = bl[m].line / E;
    fa[m] = touched ? (box_slot(D, gx, ry, rz) | (sh ? 1 << 12 : 0)) : -1;
    fs[m] = sh ? bl[m].slot_base + __popcll(bl[m].shared & (gbit - 1)) : gx + s1 * ry + s2 * rz;
  }
  if (accumulate) {  // exclusive nodes start from y: their accumulator slot is seeded with it
#pragma unroll
    for (int m = 0; m < kLines; ++m) yv[m] = y[box_base + (fa[m] >= 0 && fa[m] < (1 << 12) ? fs[m] : 0)];
  }
  const int f = tid / TL, t = tid - f * TL;
  const bool in_block = tid < NT;
  const int t1 = (D == 3) ? t % K : t;
  const int t2 = (D == 3) ? t / K : 0;
  double pj[k];
#pragma unroll
  for (int j = 0; j < k; ++j) pj[j] = 0.0;

  // The brick's visits are staged in LDS, and the gather of batch b+1 is issued before the work on
  // batch b, so global-memory latency overlaps the contractions, barriers and LDS accumulation.
  __shared__ Visit svis[kVisitChunk];
  if (tid < nv0) svis[tid] = v_first;
  __syncthreads();  // also orders the zeroing of acc before the seeding below
  for (int vc = 0; vc < visit_count; vc += kVisitChunk) {
    const int nv = min(visit_count - vc, kVisitChunk);
    if (vc > 0) {
      __syncthreads();
      for (int i = tid; i < nv; i += kBoxThreads) svis[i] = visits[visit_first + vc + i];
      __syncthreads();
    }
    VisitPrep nxt = prep_visit<D, K>(in_block && f < nv ? svis[f] : Visit(0), in_block && f < nv, t1, t2, s0, s1,
                                     s2, o0, o1, o2);
    T lnext[NN], unext[NN];
#pragma unroll
    for (int i = 0; i < NN; ++i) {
      lnext[i] = x[nxt.base + i * nxt.sn];
      if (VJP) unext[i] = u2[nxt.base + i * nxt.sn];
    }
    if (vc == 0 && accumulate) {  // seed; the barrier after the first contraction orders it before the adds
#pragma unroll
      for (int m = 0; m < kLines; ++m)
        if (fa[m] >= 0 && fa[m] < (1 << 12)) acc[fa[m]] = yv[m];
    }
  for (int v0 = 0; v0 < nv; v0 += FPB) {
    const VisitPrep cur = nxt;
    const bool live = cur.live, prim = cur.prim;
    const int ilo = cur.ilo, ihi = cur.ihi;
    T line[NN], uline[NN];
#pragma unroll
    for (int i = 0; i < NN; ++i) {
      line[i] = lnext[i];
      uline[i] = VJP ? unext[i] : T(0);
    }
    if (v0 + FPB < nv) {  // issue the next batch's gather
      const int vi = v0 + FPB + f;
      nxt = prep_visit<D, K>(in_block && vi < nv ? svis[vi] : Visit(0), in_block && vi < nv, t1, t2, s0, s1, s2, o0,
                             o1, o2);
#pragma unroll
      for (int i = 0; i < NN; ++i) {
        lnext[i] = x[nxt.base + i * nxt.sn];
        if (VJP) unext[i] = u2[nxt.base + i * nxt.sn];
      }
    }

    // normal contraction, folded with the reflection symmetry g_j[2k-i] = (-1)^(j+1) g_j[i]
    // (order j+1 odd in this 0-based loop: symmetric rows use the sums, antisymmetric rows the differences)
    T a[k], au[k];
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
          s = g[j * NN + k] * line[k];
          if (VJP) su = g[j * NN + k] * uline[k];
#pragma unroll
          for (int i = 0; i < k; ++i) {
            s = fma(g[j * NN + i], ev[i], s);
            if (VJP) su = fma(g[j * NN + i], eu[i], su);
          }
        } else {
          s = T(0);
#pragma unroll
          for (int i = 0; i < k; ++i) {
            s = fma(g[j * NN + i], od[i], s);
            if (VJP) su = fma(g[j * NN + i], ou[i], su);
          }
        }
        a[j] = live ? s : T(0);
        au[j] = (VJP && live && prim) ? su : T(0);
      }
    }
    if (in_block) {
#pragma unroll
      for (int j = 0; j < k; ++j) sa[(f * k + j) * TL + t] = a[j];
    }
    __syncthreads();
    // tangential masses in place: each row (column) is read and rewritten by the one thread that owns
    // it, and the barrier between the passes orders the row writes before the column reads
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
          for (int m = 0; m < K; ++m) s = fma(M[q * K + m], r[m], s);
          row[q] = s;
        }
      }
      __syncthreads();
      if (in_block && t2 < k) {
        T *col = &sa[(f * k + t2) * TL + t1];
        T r[K];
#pragma unroll
        for (int m = 0; m < K; ++m) r[m] = col[m * K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
          T s = T(0);
#pragma unroll
          for (int m = 0; m < K; ++m) s = fma(M[q * K + m], r[m], s);
          col[q * K] = s;
        }
      }
      __syncthreads();
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
          for (int m = 0; m < K; ++m) s = fma(M[q * K + m], r[m], s);
          row[q] = s;
        }
      }
      __syncthreads();
    }
    const T *res = sa;
    T cj[k];
#pragma unroll
    for (int j = 0; j < k; ++j) cj[j] = in_block ? res[(f * k + j) * TL + t] : T(0);
    if (live) {
      // expansion y_i = sum_j gs_j[i] c_j, folded: E_i from the symmetric orders, O_i from the others
      T yv[NN];
#pragma unroll
      for (int i = 0; i <= k; ++i) {
        T e = T(0), o = T(0);
#pragma unroll
        for (int j = 0; j < k; ++j) {
          if (j % 2 == 0)
            e = fma(gs[j * NN + i], cj[j], e);
          else if (i < k)
            o = fma(gs[j * NN + i], cj[j], o);
        }
        yv[i] = e + o;
        if (i < k) yv[2 * k - i] = e - o;
      }
      const int axis = cur.axis, rn = cur.rn, ra = cur.ra, rb = cur.rb;
#pragma unroll
      for (int i = 0; i < NN; ++i) {
        if (i >= ilo && i <= ihi) {
          const int xn = rn + i;
          const int bx0 = axis == 0 ? xn : ra;
          const int by = axis == 1 ? xn : (axis == 0 ? ra : rb);
          const int bz = axis == 2 ? xn : rb;
          __hip_atomic_fetch_add(&acc[box_slot(D, bx0, by, D == 3 ? bz : 0)], yv[i], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
      if (VJP && prim) {
#pragma unroll
        for (int j = 0; j < k; ++j) pj[j] += (double)au[j] * (double)cj[j];
      }
    }
    __syncthreads();  // sa / sb are reused by the next batch, acc is complete after the last
  }
  }

  // flush: exclusive nodes to y, shared ones to their halo slot (no global loads here)
#pragma unroll
  for (int m = 0; m < kLines; ++m) {
    if (fa[m] >= 0) {
      const T v = acc[fa[m] & 0xFFF];
      if (fa[m] >> 12)
        halo[fs[m]] = v;
      else
        y[box_base + fs[m]] = v;
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
    __syncthreads();
    if (tid < k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kBoxThreads / 64; ++w) s += red[w][tid];
      partial[(int64_t)bi * k + tid] = s;
    }
  }
}

#define GHOST_BOX_PARAMS                                                                                  \
  const T *__restrict__ x, const T *__restrict__ u2, T *__restrict__ y, T *__restrict__ halo,             \
      double *__restrict__ partial, const Box *__restrict__ boxes, const Visit *__restrict__ visits,      \
      const BoxLine *__restrict__ lines, const T *__restrict__ tab, int s0, int s1, int s2, int accumulate
#define GHOST_BOX_ARGS x, u2, y, halo, partial, boxes, visits, lines, tab, s0, s1, s2, accumulate

// Two blocks of 512 threads per CU need at most 128 VGPRs (4 waves per SIMD); the compiler is held to
// that where it fits without spilling (the apply up to k = 6).  The VJP and k = 7 carry more live
// values and run one block per CU instead.
template <typename T, int D, int K, bool VJP>
__global__ __launch_bounds__(kBoxThreads) __attribute__((amdgpu_waves_per_eu(4))) void box_kernel(
    GHOST_BOX_PARAMS) {
  box_body<T, D, K, VJP>(GHOST_BOX_ARGS);
}

template <typename T, int D, int K, bool VJP>
__global__ __launch_bounds__(kBoxThreads) void box_kernel_wide(GHOST_BOX_PARAMS) {
  box_body<T, D, K, VJP>(GHOST_BOX_ARGS);
}
#undef GHOST_BOX_PARAMS
#undef GHOST_BOX_ARGS

// y[node] (+)= sum of the node's halo slots, for every support node on a shared box face.
template <typename T>
__global__ void halo_kernel(T *__restrict__ y, const T *__restrict__ halo, const int64_t *__restrict__ node,
                            const int32_t *__restrict__ ptr, const int32_t *__restrict__ slot, int n, int accumulate) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= n) return;
  T s = T(0);
  for (int q = ptr[h]; q < ptr[h + 1]; ++q) s += halo[slot[q]];
  T *p = y + node[h];
  *p = accumulate ? *p + s : s;
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


template <typename T, int D, int K, bool VJP>
void launch_box(const DevPlan &p, const T *x, const T *u2, T *y, T *halo, const T *tab, bool accumulate,
                hipStream_t s) {
  const dim3 grid(p.n_boxes), block(kBoxThreads);
  if constexpr (VJP || K == 8)
    hipLaunchKernelGGL((box_kernel_wide<T, D, K, VJP>), grid, block, 0, s, x, u2, y, halo, p.vjp_partial, p.boxes,
                       p.visits, p.box_lines, tab, p.stride[0], p.stride[1], p.stride[2], (int)accumulate);
  else
    hipLaunchKernelGGL((box_kernel<T, D, K, VJP>), grid, block, 0, s, x, u2, y, halo, p.vjp_partial, p.boxes,
                       p.visits, p.box_lines, tab, p.stride[0], p.stride[1], p.stride[2], (int)accumulate);
}

template <typename T, bool VJP>
hipError_t dispatch_box(const DevPlan &p, const T *x, const T *u2, T *y, const T *tab, bool accumulate,
                        hipStream_t s) {
  if (p.n_boxes <= 0) return hipSuccess;
  T *halo = reinterpret_cast<T *>(p.halo);
  hipError_t e = hipErrorInvalidValue;
#define GHOST_BCASE(D_, K_)                                           \
  if (p.dim == D_ && p.k + 1 == K_) {                                 \
    launch_box<T, D_, K_, VJP>(p, x, u2, y, halo, tab, accumulate, s); \
    e = hipGetLastError();                                            \
  }
  GHOST_BCASE(2, 2) GHOST_BCASE(2, 3) GHOST_BCASE(2, 4) GHOST_BCASE(2, 5) GHOST_BCASE(2, 6) GHOST_BCASE(2, 7)
  GHOST_BCASE(2, 8) GHOST_BCASE(3, 2) GHOST_BCASE(3, 3) GHOST_BCASE(3, 4) GHOST_BCASE(3, 5) GHOST_BCASE(3, 6)
  GHOST_BCASE(3, 7) GHOST_BCASE(3, 8)
#undef GHOST_BCASE
  if (e != hipSuccess || p.n_halo == 0) return e;
  hipLaunchKernelGGL((halo_kernel<T>), dim3((p.n_halo + kBlockThreads - 1) / kBlockThreads), dim3(kBlockThreads), 0,
                     s, y, (const T *)halo, p.halo_node, p.halo_ptr, p.halo_slot, p.n_halo, (int)accumulate);
  return hipGetLastError();
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
  if (p.scatter == Scatter::Owner) return dispatch_box<double, false>(p, u, nullptr, y, p.tab64, accumulate, s);
  if (!accumulate) {
    hipError_t e = zero_support(p, y, s);
    if (e != hipSuccess) return e;
  }
  return run_faces<double, false>(p, u, nullptr, y, p.tab64, s);
}

hipError_t launch_apply_f32(const DevPlan &p, const float *u, float *y, bool accumulate, hipStream_t s) {
  if (p.scatter == Scatter::Owner) return dispatch_box<float, false>(p, u, nullptr, y, p.tab32, accumulate, s);
  if (!accumulate) {
    hipError_t e = zero_support(p, y, s);
    if (e != hipSuccess) return e;
  }
  return run_faces<float, false>(p, u, nullptr, y, p.tab32, s);
}

hipError_t launch_vjp(const DevPlan &p, const double *u, const double *w, double *du, double *dgamma,
                      bool accumulate, hipStream_t s) {
  const bool owner = p.scatter == Scatter::Owner;
  const int n_parts = owner ? p.n_boxes : p.n_batches;
  hipError_t e = hipSuccess;
  if (owner) {
    e = dispatch_box<double, true>(p, w, u, du, p.tab64, accumulate, s);
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
