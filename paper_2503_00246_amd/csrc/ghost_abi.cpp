// C ABI of libghost: argument checking, context ownership, uploads, error reporting.
// No C++ exception crosses this file's extern "C" functions.
#include <hip/hip_runtime_api.h>

#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ghost.h"
#include "ghost_device.h"
#include "ghost_plan.h"
#include "ghost_cg.h"

struct ghost_ctx {
  ghost::Plan plan;
  ghost::DevPlan dev;
  int device = -1;
  std::vector<double> gamma;
  std::vector<void *> allocs;         // device allocations owned by the context
  ghost::CgWork *cg = nullptr;        // lazily allocated CG workspace
  // per-kernel timing: event triples of the recorded calls since the last read (pool reused)
  bool timing = false;
  std::vector<std::array<hipEvent_t, 3>> events;
  size_t events_used = 0;
};

namespace {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int fail_hip(hipError_t e, const char *what) {
  return fail(GHOST_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Makes ctx's device current for the duration of a call and restores the caller's.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err != hipSuccess) { ok = false; return; }
    if (prev != dev) {
      err = hipSetDevice(dev);
      ok = err == hipSuccess;
    }
  }
  ~DeviceGuard() {
    int cur = -1;
    if (ok && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <typename T>
int upload(ghost_ctx *c, const T *src, size_t n, T **dst) {
  *dst = nullptr;
  if (n == 0) return GHOST_OK;
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(GHOST_ENOMEM, "hipMalloc of %zu bytes failed: %s", n * sizeof(T), hipGetErrorString(e));
  }
  c->allocs.push_back(p);
  if (src) {
    e = hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
  }
  *dst = static_cast<T *>(p);
  return GHOST_OK;
}

void free_device(ghost_ctx *c) {
  if (c->device < 0) return;
  DeviceGuard g(c->device);
  for (auto &t : c->events)
    for (hipEvent_t e : t)
      if (e) (void)hipEventDestroy(e);
  c->events.clear();
  if (c->cg) ghost::cg_free(c->cg);
  c->cg = nullptr;
  for (void *p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
}

bool finite_nonneg(const double *g, int k) {
  for (int j = 0; j < k; ++j)
    if (!std::isfinite(g[j]) || g[j] < 0) return false;
  return true;
}

// Host copy of both table buffers for the current gamma.
void host_tables(const ghost_ctx *c, std::vector<double> &t64, std::vector<float> &t32) {
  const ghost::Plan &p = c->plan;
  const int k = p.k, NN = 2 * k + 1, K = k + 1;
  t64.assign(ghost::tab_size64(k), 0.0);
  t32.assign(ghost::tab_size32(k), 0.0f);
  // h-power of each coefficient: h^{d-1-2j} for order j (derivative form), h^{d-2} for gamma_M (the
  // patch integral of h^{-2} times the extension difference, h^d times its reference value)
  const int ng = c->dev.n_gamma;
  for (int j = 0; j < ng; ++j) {
    const int e = c->dev.macro ? p.dim - 2 : p.dim - 1 - 2 * (j + 1);
    t64[ghost::tab_hscale(k) + j] = (double)powl((long double)p.h, (long double)e);
  }
  for (int i = 0; i < k * NN; ++i) {
    const int j = i / NN;
    t64[i] = p.jumps[i];
    if (j < ng) t64[ghost::tab_gs(k) + i] = (c->gamma[j] * t64[ghost::tab_hscale(k) + j]) * p.jumps[i];
  }
  for (int j = 0; j < ng; ++j) t64[ghost::tab_coef(k) + j] = c->gamma[j] * t64[ghost::tab_hscale(k) + j];
  for (int i = 0; i < K * K; ++i) t64[ghost::tab_M(k) + i] = p.mass[i];
  for (int i = 0; i < K; ++i) t64[ghost::tab_gllw(k) + i] = p.weights[i];
  for (int i = 0; i < k * k; ++i) t64[ghost::tab_mix(k) + i] = p.mix[i];
  for (int i = 0; i < ghost::tab_size32(k); ++i) t32[i] = (float)t64[i];
}

int check_apply(const ghost_ctx *ctx, const void *u, const void *y, size_t elem) {
  if (!ctx) return fail(GHOST_EINVAL, "null context");
  if (ctx->device < 0) return fail(GHOST_ESTATE, "host-only context (device = -1) cannot apply");
  if (!u || !y) return fail(GHOST_EINVAL, "null vector pointer");
  const char *a = static_cast<const char *>(u), *b = static_cast<const char *>(y);
  const size_t bytes = (size_t)ctx->plan.n_lattice * elem;
  if ((a <= b && b < a + bytes) || (b <= a && a < b + bytes))
    return fail(GHOST_EINVAL, "input and output vectors overlap");
  return GHOST_OK;
}

}  // namespace

namespace ghost {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
const DevPlan &dev_plan(const ghost_ctx *c) { return c->dev; }
const Plan &host_plan(const ghost_ctx *c) { return c->plan; }
CgWork *&cg_slot(ghost_ctx *c) { return c->cg; }
int ctx_device(const ghost_ctx *c) { return c->device; }
}  // namespace ghost

extern "C" {

const char *ghost_last_error(void) { return g_error.c_str(); }

int ghost_setup(const ghost_mesh *mesh, const ghost_levelset *ls, int k, const double *gamma, unsigned flags,
                int device, ghost_ctx **out) {
  g_error.clear();
  if (!out) return fail(GHOST_EINVAL, "out is null");
  *out = nullptr;
  if (!mesh || !ls || !gamma) return fail(GHOST_EINVAL, "null mesh, level set or gamma");
  if (mesh->dim != 2 && mesh->dim != 3) return fail(GHOST_EINVAL, "dim must be 2 or 3 (got %d)", mesh->dim);
  if (k < 1 || k > GHOST_KMAX) return fail(GHOST_EINVAL, "k must be in 1..%d (got %d)", GHOST_KMAX, k);
  for (int a = 0; a < mesh->dim; ++a) {
    if (mesh->n[a] < 2) return fail(GHOST_EINVAL, "n[%d] must be >= 2", a);
    if (mesh->n[a] > (1 << 20)) return fail(GHOST_EINVAL, "n[%d] too large", a);
    if (!std::isfinite(mesh->lo[a])) return fail(GHOST_EINVAL, "lo must be finite");
  }
  if (!(mesh->h > 0) || !std::isfinite(mesh->h)) return fail(GHOST_EINVAL, "h must be positive and finite");
  const bool macro = (flags & GHOST_MACRO_PATCH) != 0;
  const int n_gamma = macro ? 1 : k;
  if (!finite_nonneg(gamma, n_gamma)) return fail(GHOST_EINVAL, "gamma must be finite and >= 0");
  if (ls->kind == GHOST_LS_BALL) {
    if (!(ls->radius > 0) || !std::isfinite(ls->radius)) return fail(GHOST_EINVAL, "radius must be positive");
    for (int a = 0; a < mesh->dim; ++a)
      if (!std::isfinite(ls->centre[a])) return fail(GHOST_EINVAL, "centre must be finite");
  } else if (ls->kind == GHOST_LS_CELLS) {
    if (!ls->cell_class) return fail(GHOST_EINVAL, "cell_class is null");
  } else if (ls->kind == GHOST_LS_BALLS) {
    if (ls->n_balls < 1 || !ls->balls) return fail(GHOST_EINVAL, "balls: need n_balls >= 1 and a ball array");
    for (int i = 0; i < ls->n_balls; ++i) {
      const double *b = ls->balls + 4 * i;
      for (int a = 0; a < mesh->dim; ++a)
        if (!std::isfinite(b[a])) return fail(GHOST_EINVAL, "ball %d: centre must be finite", i);
      if (!(b[3] > 0) || !std::isfinite(b[3])) return fail(GHOST_EINVAL, "ball %d: radius must be positive", i);
    }
  } else {
    return fail(GHOST_EINVAL, "unknown level-set kind %d", ls->kind);
  }
  if (flags & ~(GHOST_FP64 | GHOST_FP32 | GHOST_COLOURED | GHOST_ATOMIC | GHOST_MACRO_PATCH))
    return fail(GHOST_EINVAL, "unknown flags");
  if ((flags & GHOST_COLOURED) && (flags & GHOST_ATOMIC))
    return fail(GHOST_EINVAL, "GHOST_COLOURED and GHOST_ATOMIC are exclusive");
  if (macro && (flags & (GHOST_COLOURED | GHOST_ATOMIC)))
    return fail(GHOST_EINVAL, "GHOST_MACRO_PATCH runs on the box scatter only (no GHOST_COLOURED / GHOST_ATOMIC)");
  if (device < -1) return fail(GHOST_EINVAL, "device must be >= -1");

  ghost_ctx *c = new (std::nothrow) ghost_ctx;
  if (!c) return fail(GHOST_ENOMEM, "out of host memory");
  try {
    c->gamma.assign(gamma, gamma + n_gamma);
    std::string err = ghost::build_plan(c->plan, mesh->dim, mesh->n, mesh->lo, mesh->h, k, ls->kind,
                                        ls->centre, ls->radius, ls->cell_class, ls->n_balls, ls->balls,
                                        (flags & GHOST_COLOURED) != 0);
    if (!err.empty()) {
      delete c;
      return fail(GHOST_EINVAL, "%s", err.c_str());
    }
  } catch (const std::bad_alloc &) {
    delete c;
    return fail(GHOST_ENOMEM, "out of host memory building the plan");
  } catch (...) {
    delete c;
    return fail(GHOST_EINVAL, "plan construction failed");
  }

  const ghost::Plan &p = c->plan;
  ghost::DevPlan &d = c->dev;
  d.dim = p.dim;
  d.k = p.k;
  d.macro = macro;
  d.n_gamma = n_gamma;
  d.h = p.h;
  for (int a = 0; a < 3; ++a) {
    d.stride[a] = (int32_t)p.stride[a];
    d.n[a] = p.n[a];
    d.L[a] = p.L[a];
  }
  d.n_batches = (int)p.batches.size();
  d.scatter = (flags & GHOST_COLOURED) ? ghost::Scatter::Coloured
              : (flags & GHOST_ATOMIC) ? ghost::Scatter::Atomic : ghost::Scatter::Box;
  d.n_boxes = (int)p.boxes.size();
  d.n_halo = (int)p.halo_node.size();
  d.n_halo_single = (int)p.n_halo_single;
  d.coloured = p.coloured;
  d.n_colours = p.n_colours;
  d.colour_begin = p.colour_begin.empty() ? nullptr : p.colour_begin.data();
  d.n_support_runs = (int)p.support_runs.size();
  d.n_active_runs = (int)p.active_runs.size();

  if (device >= 0) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || device >= count) {
      delete c;
      return e != hipSuccess ? fail_hip(e, "hipGetDeviceCount")
                             : fail(GHOST_EINVAL, "device %d not present (%d devices)", device, count);
    }
    c->device = device;
    DeviceGuard g(device);
    if (!g.ok) {
      c->device = -1;
      delete c;
      return fail_hip(g.err, "hipSetDevice");
    }
    std::vector<double> t64;
    std::vector<float> t32;
    host_tables(c, t64, t32);
    int rc = GHOST_OK;
    const int64_t *fb = nullptr;
    const ghost::Batch *bt = nullptr;
    const ghost::Run *sr = nullptr, *ar = nullptr;
    const int8_t *cl = nullptr;
    if (rc == GHOST_OK) rc = upload(c, p.face_base.data(), p.face_base.size(), const_cast<int64_t **>(&fb));
    if (rc == GHOST_OK) rc = upload(c, p.batches.data(), p.batches.size(), const_cast<ghost::Batch **>(&bt));
    if (rc == GHOST_OK) rc = upload(c, p.support_runs.data(), p.support_runs.size(), const_cast<ghost::Run **>(&sr));
    if (rc == GHOST_OK) rc = upload(c, p.active_runs.data(), p.active_runs.size(), const_cast<ghost::Run **>(&ar));
    if (rc == GHOST_OK) rc = upload(c, p.cls.data(), p.cls.size(), const_cast<int8_t **>(&cl));
    const ghost::CellChunk *ib = nullptr;
    if (rc == GHOST_OK)
      rc = upload(c, p.inside_chunks.data(), p.inside_chunks.size(), const_cast<ghost::CellChunk **>(&ib));
    d.inside_chunks = ib;
    for (int q = 0; q <= 8; ++q) d.inside_colour_begin[q] = p.inside_colour_begin[q];
    if (rc == GHOST_OK) rc = upload(c, t64.data(), t64.size(), &d.tab64);
    if (rc == GHOST_OK) rc = upload(c, t32.data(), t32.size(), &d.tab32);
    const ghost::Box *bxv = nullptr;
    const ghost::Visit *vv = nullptr;
    const ghost::BoxLine *rv = nullptr;
    const int64_t *hn = nullptr;
    const int32_t *hp = nullptr, *hs = nullptr;
    double *halo = nullptr;
    if (rc == GHOST_OK) rc = upload(c, p.boxes.data(), p.boxes.size(), const_cast<ghost::Box **>(&bxv));
    {
      // the box kernel copies visits and line records in 16-byte pieces: pad both arrays by one piece
      std::vector<ghost::Visit> vpad(p.visits);
      vpad.resize(vpad.size() + 2, 0);
      std::vector<ghost::BoxLine> lpad(p.box_lines);
      lpad.push_back(ghost::BoxLine{});
      if (rc == GHOST_OK) rc = upload(c, vpad.data(), vpad.size(), const_cast<ghost::Visit **>(&vv));
      if (rc == GHOST_OK) rc = upload(c, lpad.data(), lpad.size(), const_cast<ghost::BoxLine **>(&rv));
    }
    if (rc == GHOST_OK) rc = upload(c, p.halo_node.data(), p.halo_node.size(), const_cast<int64_t **>(&hn));
    if (rc == GHOST_OK) rc = upload(c, p.halo_ptr.data(), p.halo_ptr.size(), const_cast<int32_t **>(&hp));
    if (rc == GHOST_OK) rc = upload(c, p.halo_slot.data(), p.halo_slot.size(), const_cast<int32_t **>(&hs));
    if (rc == GHOST_OK) rc = upload<double>(c, nullptr, (size_t)std::max<int64_t>(1, p.n_slots), &halo);
    if (rc == GHOST_OK)
      rc = upload<double>(c, nullptr, (size_t)std::max(1, std::max(d.n_batches, d.n_boxes)) * k, &d.vjp_partial);
    const ghost::BoxSched sched0{};
    if (rc == GHOST_OK) rc = upload(c, &sched0, 1, &d.sched);
    if (rc == GHOST_OK) {
      const hipError_t ea = hipDeviceGetAttribute(&d.n_cu, hipDeviceAttributeMultiprocessorCount, device);
      if (ea != hipSuccess) rc = fail_hip(ea, "hipDeviceGetAttribute");
    }
    d.boxes = bxv;
    d.visits = vv;
    d.box_lines = rv;
    d.halo_node = hn;
    d.halo_ptr = hp;
    d.halo_slot = hs;
    d.halo = halo;
    d.face_base = fb;
    d.batches = bt;
    d.support_runs = sr;
    d.active_runs = ar;
    d.cls = cl;
  }
  *out = c;
  return GHOST_OK;
}

void ghost_destroy(ghost_ctx *ctx) {
  if (!ctx) return;
  free_device(ctx);
  delete ctx;
}

int ghost_set_gamma(ghost_ctx *ctx, const double *gamma, int gamma_on_device, void *stream) {
  if (!ctx || !gamma) return fail(GHOST_EINVAL, "null context or gamma");
  if (ctx->device < 0) return fail(GHOST_ESTATE, "host-only context");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  hipError_t e;
  if (gamma_on_device) {
    e = ghost::launch_set_gamma(ctx->dev, gamma, static_cast<hipStream_t>(stream));
  } else {
    const int ng = ctx->dev.n_gamma;
    if (!finite_nonneg(gamma, ng)) return fail(GHOST_EINVAL, "gamma must be finite and >= 0");
    ctx->gamma.assign(gamma, gamma + ng);
    ghost::GammaArg arg{};
    for (int j = 0; j < ng; ++j) arg.v[j] = gamma[j];
    e = ghost::launch_set_gamma_host(ctx->dev, arg, static_cast<hipStream_t>(stream));
  }
  return e == hipSuccess ? GHOST_OK : fail_hip(e, "set_gamma launch");
}

// The device plan of a launch: with timing on, a copy carrying the next event triple of the pool.
int launch_plan(ghost_ctx *ctx, ghost::DevPlan &out) {
  out = ctx->dev;
  if (!ctx->timing) return GHOST_OK;
  if (ctx->events_used == ctx->events.size()) {
    std::array<hipEvent_t, 3> t{};
    for (auto &e : t) {
      const hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return fail_hip(r, "hipEventCreate");
    }
    ctx->events.push_back(t);
  }
  const auto &t = ctx->events[ctx->events_used++];
  for (int i = 0; i < 3; ++i) out.ev[i] = t[i];
  return GHOST_OK;
}

int ghost_apply(ghost_ctx *ctx, const double *u, double *y, int accumulate, void *stream) {
  int rc = check_apply(ctx, u, y, sizeof(double));
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  ghost::DevPlan dp;
  if ((rc = launch_plan(ctx, dp))) return rc;
  hipError_t e = ghost::launch_apply_f64(dp, u, y, accumulate != 0, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GHOST_OK : fail_hip(e, "apply launch");
}

int ghost_apply_f32(ghost_ctx *ctx, const float *u, float *y, int accumulate, void *stream) {
  int rc = check_apply(ctx, u, y, sizeof(float));
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  ghost::DevPlan dp;
  if ((rc = launch_plan(ctx, dp))) return rc;
  hipError_t e = ghost::launch_apply_f32(dp, u, y, accumulate != 0, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GHOST_OK : fail_hip(e, "apply_f32 launch");
}

int ghost_vjp(ghost_ctx *ctx, const double *u, const double *w, double *du, double *dgamma, int accumulate_du,
              void *stream) {
  int rc = check_apply(ctx, w, du, sizeof(double));
  if (rc) return rc;
  rc = check_apply(ctx, u, du, sizeof(double));
  if (rc) return rc;
  if (!dgamma) return fail(GHOST_EINVAL, "null dgamma");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  ghost::DevPlan dp;
  if ((rc = launch_plan(ctx, dp))) return rc;
  hipError_t e = ghost::launch_vjp(dp, u, w, du, dgamma, accumulate_du != 0, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GHOST_OK : fail_hip(e, "vjp launch");
}

int ghost_set_timing(ghost_ctx *ctx, int on) {
  if (!ctx) return fail(GHOST_EINVAL, "null context");
  if (ctx->device < 0) return fail(GHOST_ESTATE, "host-only context");
  ctx->timing = on != 0;
  return GHOST_OK;
}

int ghost_kernel_times(ghost_ctx *ctx, double *main_ms, double *halo_ms, int64_t *calls) {
  if (!ctx) return fail(GHOST_EINVAL, "null context");
  if (ctx->device < 0) return fail(GHOST_ESTATE, "host-only context");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  double a = 0, b = 0;
  const size_t n = ctx->events_used;
  ctx->events_used = 0;
  for (size_t i = 0; i < n; ++i) {
    const auto &t = ctx->events[i];
    float m01 = 0, m12 = 0;
    hipError_t e = hipEventSynchronize(t[2]);
    if (e == hipSuccess) e = hipEventElapsedTime(&m01, t[0], t[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&m12, t[1], t[2]);
    if (e != hipSuccess) return fail_hip(e, "timing events");
    a += m01;
    b += m12;
  }
  if (main_ms) *main_ms = a;
  if (halo_ms) *halo_ms = b;
  if (calls) *calls = (int64_t)n;
  return GHOST_OK;
}

int ghost_diag(ghost_ctx *ctx, double *diag, int accumulate, void *stream) {
  if (!ctx || !diag) return fail(GHOST_EINVAL, "null context or diag");
  if (ctx->device < 0) return fail(GHOST_ESTATE, "host-only context");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  hipError_t e = hipSuccess;
  if (!accumulate) e = ghost::launch_zero_support(ctx->dev, diag, static_cast<hipStream_t>(stream));
  if (e == hipSuccess) e = ghost::launch_ghost_diag(ctx->dev, diag, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GHOST_OK : fail_hip(e, "diag launch");
}

extern "C++" {
template <typename T>
int face_bench(ghost_ctx *ctx, const T *in, T *out, int64_t n_faces, int reps, void *stream) {
  if (!ctx || (n_faces > 0 && (!in || !out))) return fail(GHOST_EINVAL, "null context, in or out");
  if (ctx->device < 0) return fail(GHOST_ESTATE, "host-only context");
  if (n_faces < 0 || reps < 1) return fail(GHOST_EINVAL, "need n_faces >= 0 and reps >= 1");
  if (ctx->dev.macro) return fail(GHOST_ESTATE, "the face microbenchmark runs the derivative-jump form only");
  int64_t n_p = 2 * ctx->plan.k + 1;
  for (int a = 1; a < ctx->plan.dim; ++a) n_p *= ctx->plan.k + 1;
  if (n_faces > ((int64_t)1 << 40) / n_p) return fail(GHOST_EINVAL, "n_faces too large");
  if (n_faces > 0 && (const void *)in == (const void *)out) return fail(GHOST_EINVAL, "in and out must differ");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  hipError_t e;
  if constexpr (sizeof(T) == 8)
    e = ghost::launch_face_micro(ctx->dev, in, out, n_faces, reps, static_cast<hipStream_t>(stream));
  else
    e = ghost::launch_face_micro_f32(ctx->dev, in, out, n_faces, reps, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GHOST_OK : fail_hip(e, "face_bench launch");
}
}  // extern "C++"

int ghost_cell_apply(ghost_ctx *ctx, const double *u, double *y, void *stream) {
  int rc = check_apply(ctx, u, y, sizeof(double));
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  hipError_t e = ghost::launch_cell_apply(ctx->dev, u, y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GHOST_OK : fail_hip(e, "cell_apply launch");
}

int ghost_cell_apply_f32(ghost_ctx *ctx, const float *u, float *y, void *stream) {
  int rc = check_apply(ctx, u, y, sizeof(float));
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  hipError_t e = ghost::launch_cell_apply_f32(ctx->dev, u, y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GHOST_OK : fail_hip(e, "cell_apply_f32 launch");
}

int ghost_face_bench(ghost_ctx *ctx, const double *in, double *out, int64_t n_faces, int reps, void *stream) {
  return face_bench<double>(ctx, in, out, n_faces, reps, stream);
}

int ghost_face_bench_f32(ghost_ctx *ctx, const float *in, float *out, int64_t n_faces, int reps, void *stream) {
  return face_bench<float>(ctx, in, out, n_faces, reps, stream);
}

int ghost_mass_diag(ghost_ctx *ctx, double *diag, void *stream) {
  if (!ctx || !diag) return fail(GHOST_EINVAL, "null context or diag");
  if (ctx->device < 0) return fail(GHOST_ESTATE, "host-only context");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  hipError_t e = ghost::launch_mass_diag(ctx->dev, diag, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GHOST_OK : fail_hip(e, "mass_diag launch");
}

int ghost_info(const ghost_ctx *ctx, ghost_stats *out) {
  if (!ctx || !out) return fail(GHOST_EINVAL, "null context or output");
  const ghost::Plan &p = ctx->plan;
  std::memset(out, 0, sizeof *out);
  out->dim = p.dim;
  out->k = p.k;
  out->device = ctx->device;
  out->n_colours = p.n_colours;
  for (int a = 0; a < 3; ++a) {
    out->lattice[a] = p.L[a];
    out->n_faces[a] = (int64_t)p.face_cell[a].size() / 3;
    out->n_faces_total += out->n_faces[a];
  }
  out->n_lattice = p.n_lattice;
  out->n_cells = (int64_t)p.cls.size();
  out->n_active_cells = p.n_active_cells;
  out->n_cut_cells = p.n_cut_cells;
  out->n_active_dofs = p.n_active;
  out->n_support_dofs = p.n_support;
  out->n_inside_dofs = p.n_inside;
  out->n_gamma = ctx->dev.n_gamma;
  out->n_cell_chunks = (int64_t)p.inside_chunks.size();
  out->macro = ctx->dev.macro ? 1 : 0;
  const int K = p.k + 1;
  int64_t tang = 1;
  for (int a = 1; a < p.dim; ++a) tang *= K;
  out->n_patch_dofs = (2 * p.k + 1) * tang;
  out->n_batches = (int64_t)p.batches.size();
  out->n_boxes = (int64_t)p.boxes.size();
  out->n_visits = p.n_visits;
  out->brick = p.brick;
  out->n_halo_slots = p.n_slots;
  out->n_halo_nodes = (int64_t)p.halo_node.size();
  // contraction and expansion 2k(2k+1) per tangential line, masses (d-1)k(k+1) per line; the macro-patch
  // form also couples the orders, ceil(k^2 / 2) nonzeros of H per line
  const double coupling = ctx->dev.macro ? (double)((p.k * p.k + 1) / 2) * tang : 0.0;
  out->flops_per_face =
      2.0 * (2.0 * p.k * (2 * p.k + 1) * tang + (double)(p.dim - 1) * p.k * tang * K + coupling);
  out->bytes_fp64 = 24.0 * (double)p.n_support;
  out->bytes_fp32 = 12.0 * (double)p.n_support;
  return GHOST_OK;
}

int ghost_faces(const ghost_ctx *ctx, int axis, int32_t *out, int64_t cap) {
  if (!ctx || !out) return fail(GHOST_EINVAL, "null context or output");
  if (axis < 0 || axis >= ctx->plan.dim) return fail(GHOST_EINVAL, "axis out of range");
  const auto &fc = ctx->plan.face_cell[axis];
  const int64_t nf = (int64_t)fc.size() / 3;
  if (cap < nf) return fail(GHOST_EINVAL, "capacity %lld < %lld faces", (long long)cap, (long long)nf);
  for (int64_t f = 0; f < nf; ++f) {
    out[4 * f + 0] = fc[3 * f + 0];
    out[4 * f + 1] = fc[3 * f + 1];
    out[4 * f + 2] = fc[3 * f + 2];
    out[4 * f + 3] = ctx->plan.face_colour[axis][f];
  }
  return GHOST_OK;
}

int ghost_cell_chunks(const ghost_ctx *ctx, int64_t *out, int64_t cap) {
  if (!ctx || !out) return fail(GHOST_EINVAL, "null context or output");
  const ghost::Plan &p = ctx->plan;
  const int64_t n = (int64_t)p.inside_chunks.size();
  if (cap < n) return fail(GHOST_EINVAL, "capacity %lld < %lld chunks", (long long)cap, (long long)n);
  for (int col = 0; col < 8; ++col)
    for (int64_t i = p.inside_colour_begin[col]; i < p.inside_colour_begin[col + 1]; ++i) {
      out[3 * i] = p.inside_chunks[i].base;
      out[3 * i + 1] = p.inside_chunks[i].count;
      out[3 * i + 2] = col;
    }
  return GHOST_OK;
}

int ghost_box_layout(const ghost_ctx *ctx, int32_t *boxes, int64_t box_cap, uint64_t *visits, int64_t visit_cap,
                     int64_t *runs, int64_t run_cap) {
  if (!ctx) return fail(GHOST_EINVAL, "null context");
  const ghost::Plan &p = ctx->plan;
  if (boxes) {
    if (box_cap < (int64_t)p.boxes.size()) return fail(GHOST_EINVAL, "box capacity too small");
    for (size_t i = 0; i < p.boxes.size(); ++i) {
      const ghost::Box &b = p.boxes[i];
      int32_t *o = boxes + 7 * i;
      for (int a = 0; a < 3; ++a) o[a] = b.org[a];
      o[3] = b.visit_first;
      o[4] = b.visit_count;
      o[5] = b.run_first;
      o[6] = b.run_count;
    }
  }
  if (visits) {
    if (visit_cap < (int64_t)p.visits.size()) return fail(GHOST_EINVAL, "visit capacity too small");
    std::memcpy(visits, p.visits.data(), p.visits.size() * sizeof(uint64_t));
  }
  if (runs) {
    if (run_cap < (int64_t)p.box_runs.size()) return fail(GHOST_EINVAL, "run capacity too small");
    for (size_t i = 0; i < p.box_runs.size(); ++i) {
      runs[4 * i] = p.box_runs[i].start;
      runs[4 * i + 1] = p.box_runs[i].acc;
      runs[4 * i + 2] = p.box_runs[i].len;
      runs[4 * i + 3] = p.box_runs[i].slot;
    }
  }
  return GHOST_OK;
}

int ghost_tables(const ghost_ctx *ctx, double *jumps, double *mass, double *nodes, double *weights) {
  if (!ctx) return fail(GHOST_EINVAL, "null context");
  const ghost::Plan &p = ctx->plan;
  if (jumps) std::memcpy(jumps, p.jumps.data(), p.jumps.size() * sizeof(double));
  if (mass) std::memcpy(mass, p.mass.data(), p.mass.size() * sizeof(double));
  if (nodes) std::memcpy(nodes, p.nodes.data(), p.nodes.size() * sizeof(double));
  if (weights) std::memcpy(weights, p.weights.data(), p.weights.size() * sizeof(double));
  return GHOST_OK;
}

int ghost_cg(ghost_ctx *ctx, const double *b, double *x, const ghost_cg_opts *opts, ghost_cg_result *res,
             void *stream) {
  if (!ctx || !b || !x || !opts || !res) return fail(GHOST_EINVAL, "null argument");
  if (ctx->device < 0) return fail(GHOST_ESTATE, "host-only context");
  if (b == x) return fail(GHOST_EINVAL, "b and x must differ");
  if (opts->mode != GHOST_CG_FP64 && opts->mode != GHOST_CG_MIXED) return fail(GHOST_EINVAL, "unknown CG mode");
  if (opts->precond != GHOST_CG_NONE && opts->precond != GHOST_CG_JACOBI)
    return fail(GHOST_EINVAL, "unknown CG preconditioner");
  if (!(opts->tol > 0) || opts->max_iter < 1) return fail(GHOST_EINVAL, "tol must be > 0 and max_iter >= 1");
  if (opts->mode == GHOST_CG_MIXED && !(opts->inner_tol > 0 && opts->inner_tol < 1))
    return fail(GHOST_EINVAL, "inner_tol must be in (0, 1)");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail_hip(g.err, "hipSetDevice");
  try {
    return ghost::cg_solve(ctx, b, x, *opts, *res, static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc &) {
    return fail(GHOST_ENOMEM, "out of host memory in CG");
  } catch (...) {
    return fail(GHOST_EINVAL, "CG failed");
  }
}

}  // extern "C"
