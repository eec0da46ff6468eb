// Conjugate gradients on A x = b, A = M + G over the active lattice nodes, with all
// vector operations in this file's kernels and every scalar (alpha, beta, residual
// norms) kept on the device; the host reads one double per iteration for the stopping
// test.  The paper leaves the solver open (§1, last paragraphs); this driver is the
// linear-solve workload around the ghost-penalty apply.
//
// FP64 mode: plain CG from x = 0.  The recursive residual is replaced by the true one,
// b - A x, every check_every iterations and whenever it meets the tolerance; the solve
// stops on the true residual.  With the Jacobi preconditioner (1 / diag(M + G), built per
// solve) the CG is the preconditioned one and the true residual is tested every
// check_every iterations.
// Mixed mode: outer refinement in FP64 (true residual r = b - A x with the FP64 apply,
// x += e), inner CG on A e = r with FP32 vectors, FP32 ghost apply and FP32 mass, and
// FP64 dot products and scalars, run until its residual drops by inner_tol.
//
// Vectors live on the lattice; kernels visit only the active nodes, cut into segments
// of at most 256 consecutive nodes.  Each wavefront takes segments in a grid-stride loop over a
// grid capped at kMaxBlocks workgroups (enough to fill the device), so that a dot product leaves at
// most kMaxBlocks partial sums for its one-block reduction.
// The host reads the recursive residual every kPoll iterations only, so that the stream is not drained
// every iteration (a solve may run up to kPoll - 1 iterations past its recursive stopping point).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "ghost_cg.h"

namespace ghost {

namespace {
constexpr int kSegLen = 256;
constexpr int kPoll = 8;
constexpr int kSegPerBlock = kBlockThreads / 64;
constexpr int kMaxBlocks = 2048;
enum { S_RR = 0, S_PQ, S_ALPHA, S_BETA, S_TMP, S_COUNT = 8 };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Per-block partial of a dot product, fixed reduction order.
__device__ __forceinline__ void block_partial(double v, double *partial) {
  __shared__ double red[kSegPerBlock];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSegPerBlock; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

// f(j) for every active node j; the wave's lanes take consecutive nodes of a segment.
template <typename F>
__device__ __forceinline__ void for_active(const Run *__restrict__ segs, int n_segs, F f) {
  const int lane = threadIdx.x & 63;
  for (int seg = blockIdx.x * kSegPerBlock + (threadIdx.x >> 6); seg < n_segs; seg += gridDim.x * kSegPerBlock) {
    const Run sg = segs[seg];
    for (int i = lane; i < sg.len; i += 64) f(sg.start + i);
  }
}

// With a preconditioner, z = dinv * r (Jacobi); without one (dinv null), z = r.
template <typename T>
__device__ __forceinline__ T precond(const T *dinv, int64_t j, T r) {
  return dinv ? dinv[j] * r : r;
}

// x = 0, r = (T) src, p = z; partial <r, z>
template <typename T>
__global__ void start_kernel(const Run *segs, int n_segs, const double *src, T *x, T *r, T *p, const T *dinv,
                             double *partial) {
  double acc = 0.0;
  for_active(segs, n_segs, [&](int64_t j) {
    const T v = (T)src[j];
    const T z = precond(dinv, j, v);
    x[j] = T(0);
    r[j] = v;
    p[j] = z;
    acc += (double)v * (double)z;
  });
  block_partial(acc, partial);
}

// Optionally x += alpha p (the previous step's update of x, deferred to this pass, which reads p anyway),
// optionally p = z + beta p, then q = mdiag * p; partial <p, q>, the mass part of <p, A p>.
template <typename T>
__global__ void pq_kernel(const Run *segs, int n_segs, T *x, T *p, const T *r, T *q, const T *mdiag, const T *dinv,
                          const double *scal, int update_p, int update_x, double *partial) {
  const T beta = (T)scal[S_BETA], alpha = (T)scal[S_ALPHA];
  double acc = 0.0;
  for_active(segs, n_segs, [&](int64_t j) {
    T pv = p[j];
    if (update_x) x[j] += alpha * pv;
    if (update_p) {
      pv = precond(dinv, j, r[j]) + beta * pv;
      p[j] = pv;
    }
    const T qv = mdiag[j] * pv;
    q[j] = qv;
    acc += (double)pv * (double)qv;
  });
  block_partial(acc, partial);
}

// partial <p, q - mdiag p> over the support nodes: the ghost part of <p, A p> (G p vanishes elsewhere),
// with mdiag p rounded as pq_kernel rounded it into q.
template <typename T>
__global__ void ghost_dot_kernel(const Run *segs, int n_segs, const T *p, const T *q, const T *mdiag,
                                 double *partial) {
  double acc = 0.0;
  for_active(segs, n_segs, [&](int64_t j) {
    const T pv = p[j];
    const T mp = mdiag[j] * pv;
    acc += (double)pv * ((double)q[j] - (double)mp);
  });
  block_partial(acc, partial);
}

// x += alpha p (the deferred update, when the solve needs x)
template <typename T>
__global__ void axpy_kernel(const Run *segs, int n_segs, T *x, const T *p, const double *scal) {
  const T alpha = (T)scal[S_ALPHA];
  for_active(segs, n_segs, [&](int64_t j) { x[j] += alpha * p[j]; });
}

template <typename T>
__global__ void dot_kernel(const Run *segs, int n_segs, const T *a, const T *b, double *partial) {
  double acc = 0.0;
  for_active(segs, n_segs, [&](int64_t j) {
    acc += (double)a[j] * (double)b[j];
  });
  block_partial(acc, partial);
}

// r -= alpha q; partial <r, z> (x += alpha p is deferred to the next pq_kernel or axpy_kernel)
template <typename T>
__global__ void xr_kernel(const Run *segs, int n_segs, T *r, const T *q, const T *dinv, const double *scal,
                          double *partial) {
  const T alpha = (T)scal[S_ALPHA];
  double acc = 0.0;
  for_active(segs, n_segs, [&](int64_t j) {
    const T rv = r[j] - alpha * q[j];
    r[j] = rv;
    acc += (double)rv * (double)precond(dinv, j, rv);
  });
  block_partial(acc, partial);
}

// partial <r, dinv r>
__global__ void rz_kernel(const Run *segs, int n_segs, const double *r, const double *dinv, double *partial) {
  double acc = 0.0;
  for_active(segs, n_segs, [&](int64_t j) {
    acc += r[j] * dinv[j] * r[j];
  });
  block_partial(acc, partial);
}

// d = 1 / d on the active nodes (the Jacobi preconditioner from the diagonal of A), and its FP32 copy
__global__ void invert_kernel(const Run *segs, int n_segs, double *d, float *d32) {
  for_active(segs, n_segs, [&](int64_t j) {
    const double v = 1.0 / d[j];
    d[j] = v;
    d32[j] = (float)v;
  });
}

// q = mdiag * x (FP64), the mass part of A x
__global__ void mass_kernel(const Run *segs, int n_segs, const double *x, const double *mdiag, double *q) {
  for_active(segs, n_segs, [&](int64_t j) {
    q[j] = mdiag[j] * x[j];
  });
}

// r = b - q; partial <r, r>
__global__ void residual_kernel(const Run *segs, int n_segs, const double *b, const double *q, double *r,
                                double *partial) {
  double acc = 0.0;
  for_active(segs, n_segs, [&](int64_t j) {
    const double v = b[j] - q[j];
    r[j] = v;
    acc += v * v;
  });
  block_partial(acc, partial);
}

// x += (double) e; also zero x (init) when mode == 1
__global__ void add_kernel(const Run *segs, int n_segs, double *x, const float *e, int zero) {
  for_active(segs, n_segs, [&](int64_t j) {
    x[j] = zero ? 0.0 : x[j] + (double)e[j];
  });
}

__global__ void cast_kernel(const Run *segs, int n_segs, const double *a, float *b) {
  for_active(segs, n_segs, [&](int64_t j) {
    b[j] = (float)a[j];
  });
}

// mode 0: scal[RR] = s; 1: scal[PQ] = s, scal[ALPHA] = scal[RR] / s;
// 2: scal[BETA] = s / scal[RR], scal[RR] = s; 3: scal[TMP] = s  (a zero denominator gives 0)
// (the partial sums of two arrays: n of `partial` and n2 of `partial2`)
__global__ void reduce_kernel(const double *partial, int n, const double *partial2, int n2, double *scal, int mode) {
  __shared__ double red[kBlockThreads];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < n; i += kBlockThreads) s += partial[i];
  for (int i = tid; i < n2; i += kBlockThreads) s += partial2[i];
  red[tid] = s;
  __syncthreads();
  for (int w = kBlockThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    const double v = red[0];
    if (mode == 0) {
      scal[S_RR] = v;
    } else if (mode == 1) {
      // a step after exact convergence has p = 0: alpha = 0 keeps x and r instead of 0 / 0
      scal[S_PQ] = v;
      scal[S_ALPHA] = v != 0.0 ? scal[S_RR] / v : 0.0;
    } else if (mode == 2) {
      const double rr = scal[S_RR];
      scal[S_BETA] = rr != 0.0 ? v / rr : 0.0;
      scal[S_RR] = v;
    } else {
      scal[S_TMP] = v;
    }
  }
}


}  // namespace


struct CgWork {
  Run *segs = nullptr;
  int n_segs = 0, n_blocks = 0;
  Run *ssegs = nullptr;  // support nodes (G p vanishes elsewhere), cut like the active ones
  int n_ssegs = 0, n_sblocks = 0;
  double *partial2 = nullptr;
  double *mdiag = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *scal = nullptr, *partial = nullptr;
  float *mdiag32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *e32 = nullptr;
  double *dinv = nullptr;  // Jacobi preconditioner 1 / diag(M + G), rebuilt per preconditioned solve
  float *dinv32 = nullptr;
  double *host = nullptr;  // pinned, S_COUNT doubles
  std::vector<void *> allocs;
};

void cg_free(CgWork *w) {
  if (!w) return;
  for (void *p : w->allocs) (void)hipFree(p);
  if (w->host) (void)hipHostFree(w->host);
  delete w;
}

namespace {

template <typename T>
hipError_t alloc(CgWork *w, T **p, size_t n) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(T));
  if (e != hipSuccess) return e;
  w->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return hipSuccess;
}

hipError_t cg_init(ghost_ctx *ctx, CgWork **out, hipStream_t s) {
  const Plan &pl = host_plan(ctx);
  const DevPlan &dp = dev_plan(ctx);
  CgWork *w = new CgWork;
  std::vector<Run> segs;
  for (const Run &r : pl.active_runs)
    for (int32_t o = 0; o < r.len; o += kSegLen) segs.push_back(Run{r.start + o, std::min(kSegLen, r.len - o), 0});
  w->n_segs = (int)segs.size();
  w->n_blocks = std::min(kMaxBlocks, std::max(1, (w->n_segs + kSegPerBlock - 1) / kSegPerBlock));
  std::vector<Run> ssegs;
  for (const Run &r : pl.support_runs)
    for (int32_t o = 0; o < r.len; o += kSegLen) ssegs.push_back(Run{r.start + o, std::min(kSegLen, r.len - o), 0});
  w->n_ssegs = (int)ssegs.size();
  w->n_sblocks = std::min(kMaxBlocks, std::max(1, (w->n_ssegs + kSegPerBlock - 1) / kSegPerBlock));
  const size_t n = (size_t)pl.n_lattice;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = alloc(w, &w->segs, std::max<size_t>(1, segs.size()));
  if (e == hipSuccess && !segs.empty())
    e = hipMemcpy(w->segs, segs.data(), segs.size() * sizeof(Run), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = alloc(w, &w->ssegs, std::max<size_t>(1, ssegs.size()));
  if (e == hipSuccess && !ssegs.empty())
    e = hipMemcpy(w->ssegs, ssegs.data(), ssegs.size() * sizeof(Run), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = alloc(w, &w->partial2, (size_t)w->n_sblocks);
  if (e == hipSuccess) e = alloc(w, &w->mdiag, n);
  if (e == hipSuccess) e = alloc(w, &w->r, n);
  if (e == hipSuccess) e = alloc(w, &w->p, n);
  if (e == hipSuccess) e = alloc(w, &w->q, n);
  if (e == hipSuccess) e = alloc(w, &w->scal, S_COUNT);
  if (e == hipSuccess) e = alloc(w, &w->partial, (size_t)w->n_blocks);
  if (e == hipSuccess) e = alloc(w, &w->mdiag32, n);
  if (e == hipSuccess) e = alloc(w, &w->r32, n);
  if (e == hipSuccess) e = alloc(w, &w->p32, n);
  if (e == hipSuccess) e = alloc(w, &w->q32, n);
  if (e == hipSuccess) e = alloc(w, &w->e32, n);
  if (e == hipSuccess) e = alloc(w, &w->dinv, n);
  if (e == hipSuccess) e = alloc(w, &w->dinv32, n);
  if (e == hipSuccess) e = hipHostMalloc((void **)&w->host, S_COUNT * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = launch_mass_diag(dp, w->mdiag, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(cast_kernel, dim3(w->n_blocks), dim3(kBlockThreads), 0, s, w->segs, w->n_segs,
                       (const double *)w->mdiag, w->mdiag32);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    cg_free(w);
    return e;
  }
  *out = w;
  return hipSuccess;
}

struct Runner {
  const DevPlan &dp;
  CgWork *w;
  hipStream_t s;
  hipError_t err = hipSuccess;
  dim3 grid, block{kBlockThreads};
  Runner(const DevPlan &d, CgWork *w_, hipStream_t s_) : dp(d), w(w_), s(s_), grid(w_->n_blocks) {}
  void reduce(int mode, bool with_ghost_dot = false) {
    if (err != hipSuccess) return;
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kBlockThreads), 0, s, w->partial, w->n_blocks,
                       (const double *)w->partial2, with_ghost_dot ? w->n_sblocks : 0, w->scal, mode);
    err = hipGetLastError();
  }
  // <p, A p> into the reduction of mode 1 (alpha): the mass part from pq_kernel, the ghost part here
  template <typename T>
  void ghost_dot(const T *p, const T *q, const T *mdiag) {
    if (err != hipSuccess) return;
    hipLaunchKernelGGL(ghost_dot_kernel<T>, dim3(w->n_sblocks), block, 0, s, w->ssegs, w->n_ssegs, p, q, mdiag,
                       w->partial2);
    err = hipGetLastError();
    reduce(1, true);
  }
  template <typename T>
  void flush_x(T *x, const T *p) {
    if (err != hipSuccess) return;
    hipLaunchKernelGGL(axpy_kernel<T>, grid, block, 0, s, w->segs, w->n_segs, x, p, (const double *)w->scal);
    err = hipGetLastError();
  }
  void check() {
    if (err == hipSuccess) err = hipGetLastError();
  }
  double read(int idx) {
    if (err != hipSuccess) return NAN;
    err = hipMemcpyAsync(w->host, w->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    return err == hipSuccess ? w->host[idx] : NAN;
  }
  // r = b - A x (FP64); scal[RR] = <r, z> for the next CG step (z = dinv r, or r); returns |r|^2
  double true_residual(const double *b, const double *x, double *r, const double *dinv) {
    hipLaunchKernelGGL(mass_kernel, grid, block, 0, s, w->segs, w->n_segs, x, (const double *)w->mdiag, w->q);
    check();
    if (err == hipSuccess) err = launch_apply_f64(dp, x, w->q, true, s);
    hipLaunchKernelGGL(residual_kernel, grid, block, 0, s, w->segs, w->n_segs, b, (const double *)w->q, r,
                       w->partial);
    check();
    reduce(3);
    if (dinv) {
      hipLaunchKernelGGL(rz_kernel, grid, block, 0, s, w->segs, w->n_segs, (const double *)r, dinv, w->partial);
      check();
    }
    reduce(0);
    return read(S_TMP);
  }
};

}  // namespace

int cg_solve(ghost_ctx *ctx, const double *b, double *x, const ghost_cg_opts &opts, ghost_cg_result &res,
             hipStream_t s) {
  res = ghost_cg_result{0, 0, 0, NAN};
  CgWork *&slot = cg_slot(ctx);
  if (!slot) {
    hipError_t e = cg_init(ctx, &slot, s);
    if (e != hipSuccess) {
      slot = nullptr;
      return set_error(e == hipErrorOutOfMemory ? GHOST_ENOMEM : GHOST_EHIP, hipGetErrorString(e));
    }
  }
  CgWork *w = slot;
  const DevPlan &dp = dev_plan(ctx);
  Runner R(dp, w, s);
  const dim3 grid(w->n_blocks), block(kBlockThreads);

  // |b|
  hipLaunchKernelGGL(dot_kernel<double>, grid, block, 0, s, w->segs, w->n_segs, b, b, w->partial);
  R.check();
  R.reduce(3);
  const double bnorm = std::sqrt(R.read(S_TMP));
  if (R.err != hipSuccess) return set_error(GHOST_EHIP, hipGetErrorString(R.err));
  const double target = opts.tol * bnorm;
  int it = 0;

  // Jacobi: dinv = 1 / (mass diagonal + diagonal of G) on the active nodes
  const bool jac = opts.precond == GHOST_CG_JACOBI;
  const double *dinv = jac ? w->dinv : nullptr;
  const float *dinv32 = jac ? w->dinv32 : nullptr;
  if (jac && R.err == hipSuccess) {
    R.err = hipMemcpyAsync(w->dinv, w->mdiag, (size_t)host_plan(ctx).n_lattice * sizeof(double),
                           hipMemcpyDeviceToDevice, s);
    if (R.err == hipSuccess) R.err = launch_ghost_diag(dp, w->dinv, s);
    hipLaunchKernelGGL(invert_kernel, grid, block, 0, s, w->segs, w->n_segs, w->dinv, w->dinv32);
    R.check();
  }

  if (opts.mode == GHOST_CG_FP64) {
    hipLaunchKernelGGL(start_kernel<double>, grid, block, 0, s, w->segs, w->n_segs, b, x, w->r, w->p, dinv,
                       w->partial);
    R.check();
    R.reduce(0);
    double rr = R.read(S_RR);  // <r, z>
    double rr_true = jac ? bnorm * bnorm : rr;
    const int every = opts.check_every > 0 ? opts.check_every : 50;
    bool update_p = false, x_pending = false;  // x_pending: x still lacks alpha p of the last step
    while (R.err == hipSuccess && std::sqrt(rr_true) > target && it < opts.max_iter) {
      hipLaunchKernelGGL(pq_kernel<double>, grid, block, 0, s, w->segs, w->n_segs, x, w->p, (const double *)w->r,
                         w->q, (const double *)w->mdiag, dinv, (const double *)w->scal, (int)update_p,
                         (int)x_pending, w->partial);
      R.check();
      x_pending = false;
      if (R.err == hipSuccess) R.err = launch_apply_f64(dp, w->p, w->q, true, s);
      R.ghost_dot<double>(w->p, w->q, w->mdiag);
      hipLaunchKernelGGL(xr_kernel<double>, grid, block, 0, s, w->segs, w->n_segs, w->r, (const double *)w->q, dinv,
                         (const double *)w->scal, w->partial);
      R.check();
      x_pending = true;
      R.reduce(2);
      update_p = true;
      ++it;
      const bool poll = !jac && (it % kPoll == 0 || it >= opts.max_iter);
      if (poll) {
        rr = R.read(S_RR);  // without a preconditioner <r, z> = |r|^2: test the recursive residual
        rr_true = rr;
      }
      if ((poll && std::sqrt(rr) <= target) || it % every == 0) {
        // replace the recursive residual by the true one (the search direction is kept)
        R.flush_x(x, (const double *)w->p);
        x_pending = false;
        rr_true = R.true_residual(b, x, w->r, dinv);
      }
    }
    if (x_pending) R.flush_x(x, (const double *)w->p);
    res.outer = 1;
  } else {
    hipLaunchKernelGGL(add_kernel, grid, block, 0, s, w->segs, w->n_segs, x, (const float *)nullptr, 1);
    R.check();
    while (R.err == hipSuccess) {
      const double rr_true = R.true_residual(b, x, w->r, nullptr);
      if (!(std::sqrt(rr_true) > target) || it >= opts.max_iter) break;
      // inner FP32 CG on A e = r
      hipLaunchKernelGGL(start_kernel<float>, grid, block, 0, s, w->segs, w->n_segs, (const double *)w->r, w->e32,
                         w->r32, w->p32, dinv32, w->partial);
      R.check();
      R.reduce(0);
      double rr = R.read(S_RR);
      const double inner_target = opts.inner_tol * std::sqrt(rr);
      bool update_p = false, e_pending = false;  // e_pending: e still lacks alpha p of the last step
      while (R.err == hipSuccess && std::sqrt(rr) > inner_target && it < opts.max_iter) {
        hipLaunchKernelGGL(pq_kernel<float>, grid, block, 0, s, w->segs, w->n_segs, w->e32, w->p32,
                           (const float *)w->r32, w->q32, (const float *)w->mdiag32, dinv32, (const double *)w->scal,
                           (int)update_p, (int)e_pending, w->partial);
        R.check();
        e_pending = false;
        if (R.err == hipSuccess) R.err = launch_apply_f32(dp, w->p32, w->q32, true, s);
        R.ghost_dot<float>(w->p32, w->q32, w->mdiag32);
        hipLaunchKernelGGL(xr_kernel<float>, grid, block, 0, s, w->segs, w->n_segs, w->r32, (const float *)w->q32,
                           dinv32, (const double *)w->scal, w->partial);
        R.check();
        e_pending = true;
        R.reduce(2);
        update_p = true;
        ++it;
        if (it % kPoll == 0 || it >= opts.max_iter) {
          rr = R.read(S_RR);
          if (!std::isfinite(rr)) break;
        }
      }
      if (e_pending) R.flush_x(w->e32, (const float *)w->p32);
      hipLaunchKernelGGL(add_kernel, grid, block, 0, s, w->segs, w->n_segs, x, (const float *)w->e32, 0);
      R.check();
      ++res.outer;
    }
  }
  if (R.err != hipSuccess) return set_error(GHOST_EHIP, hipGetErrorString(R.err));
  const double rr_final = R.true_residual(b, x, w->r, nullptr);
  if (R.err != hipSuccess) return set_error(GHOST_EHIP, hipGetErrorString(R.err));
  res.iterations = it;
  res.rel_residual = bnorm > 0 ? std::sqrt(rr_final) / bnorm : 0.0;
  res.converged = res.rel_residual <= opts.tol;
  return GHOST_OK;
}

}  // namespace ghost
