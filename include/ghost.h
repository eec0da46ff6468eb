/*
 * ghost.h -- C ABI of libghost, the MI355X (gfx950) matrix-free ghost-penalty operator.
 *
 * Operation (paper "Matrix-Free Ghost Penalty Evaluation via Tensor Product
 * Factorization", §2.2 and §2.4):
 *
 *   y = G(gamma) u,   u^T G v = sum_{F in F_h} sum_{j=1..k} gamma_j (d^j_n u, d^j_n v)_F
 *
 * with jumps [.] across the face F, continuous Q_k Lagrange elements on GLL nodes,
 * F_h = interior faces between two active cells at least one of which is cut by the
 * level set (Fig. 1).  Each face matrix is applied in factored form (§2.4, the
 * summed-penalty equation; §2.5.1): a rank-k 1D penalty along the normal and the
 * exact 1D mass matrix along every tangential axis, O(k^{d+1}) per face.
 *
 * gamma_j carries every scalar of the paper's g_F; the paper's choice is
 * gamma_j = gamma_A h^{2j-1} / (j!)^2, gamma_A applied once.
 *
 * Also: the macro-patch stabilisation in place of G (GHOST_MACRO_PATCH, §2.2), the Laplacian on the
 * cells the boundary does not cut (ghost_cell_apply, §2.1), conjugate gradients on M + G (ghost_cg),
 * and a single-face microbenchmark (ghost_face_bench, §3).
 *
 * Vectors live on the full node lattice: L_a = k*n_a + 1 nodes per axis, node
 * multi-index I, linear index I_0 + L_0 I_1 + L_0 L_1 I_2 (x fastest, §2.4).
 * Entries outside the support (the union of all face patches) are neither read
 * nor written by the apply.
 *
 * Conventions for every entry point:
 *   - return 0 on success or a negative GHOST_E* code; ghost_last_error() then
 *     returns a thread-local message for the failing call.  No C++ exception
 *     crosses this interface.
 *   - vector arguments are DEVICE pointers on the context's device, owned by the
 *     caller; the library never frees or retains them past the call.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.  Apply and
 *     VJP calls are asynchronous on that stream, allocate nothing and never
 *     synchronise the host.  A context must not be used on two streams at once
 *     (its internal workspaces are shared).
 *   - kernel faults surface at the caller's next synchronisation, as with any
 *     asynchronous HIP call.
 */
#ifndef GHOST_H
#define GHOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GHOST_OK 0
#define GHOST_EINVAL (-1) /* bad argument */
#define GHOST_ENOMEM (-2) /* host or device allocation failed */
#define GHOST_EHIP (-3)   /* HIP runtime error (message carries hipGetErrorString) */
#define GHOST_ESTATE (-4) /* call not valid for this context (e.g. host-only plan) */

#define GHOST_KMAX 7

/* level-set kinds */
#define GHOST_LS_BALL 0  /* phi = radius - |x - centre| (> 0 inside, §2) */
#define GHOST_LS_CELLS 1 /* caller-provided cell classes */
#define GHOST_LS_BALLS 2 /* union of balls, phi = max_i (r_i - |x - c_i|) (the multiple-ball problem, §3) */

/* cell classes */
#define GHOST_OUTSIDE 0
#define GHOST_INSIDE 1
#define GHOST_CUT 2

/* ghost_setup flags */
#define GHOST_FP64 1u     /* accepted for clarity; both precisions are always built */
#define GHOST_FP32 2u
#define GHOST_COLOURED 4u /* scatter strategy: face-parallel, plain read-modify-write per race-free colour */
#define GHOST_ATOMIC 8u   /* scatter strategy: face-parallel, hardware FP64/FP32 atomics */
/* Macro-patch stabilisation (§2.2, the alternative to the derivative jumps with the same tensor-product
 * structure) in place of the ghost penalty:
 *   u^T S v = sum_{F in F_h} gamma_M h^-2 integral over the patch K_1 u K_2 of F of
 *             (E_1 u - E_2 u)(E_1 v - E_2 v),
 * E_i u the polynomial extension of u restricted to cell K_i.  One coefficient gamma_M (gamma, set_gamma
 * and the VJP's dgamma then have length 1).  Applied in the same rank-k form, with the k derivative
 * orders coupled by a fixed k x k matrix.  Box scatter only: not combinable with GHOST_COLOURED or
 * GHOST_ATOMIC. */
#define GHOST_MACRO_PATCH 16u
/* With neither flag the default box scatter is used: the cells are cut into bricks; a workgroup
 * applies every face with a cell in its brick (expanding only into the brick's cells), sums the
 * contributions over the brick's node box in LDS, writes nodes no other box contains straight to y
 * and passes nodes on shared box faces through halo slots that a second kernel adds into y.  No
 * global atomics; y needs no prior zeroing. */

typedef struct ghost_ctx ghost_ctx;

typedef struct {
  int dim;       /* 2 or 3 */
  int n[3];      /* cells per axis, each >= 2 (n[2] ignored when dim == 2) */
  double lo[3];  /* lower corner of the box */
  double h;      /* cell side (> 0, finite); cells are squares / cubes (§2) */
} ghost_mesh;

/* Cell classes from a level set.  Ball: a cell is active when it meets the open ball and inside when
 * it lies in the closed ball (exact distances; cut = active and not inside).  Union of balls: active
 * when it meets some open ball, inside when it lies in some closed ball, cut otherwise when active (a
 * cell that only the union of several balls covers counts as cut). */
typedef struct {
  int kind;                      /* GHOST_LS_BALL, GHOST_LS_CELLS or GHOST_LS_BALLS */
  double centre[3];              /* ball only */
  double radius;                 /* ball only, > 0 */
  const signed char *cell_class; /* cells only: HOST array of n0*n1(*n2) classes, x fastest */
  int n_balls;                   /* balls only: >= 1 */
  const double *balls;           /* balls only: HOST array of n_balls x (c0, c1, c2, r), c2 ignored in 2D,
                                    r > 0; read during ghost_setup only */
} ghost_levelset;

typedef struct {
  int dim, k;
  int device;                 /* -1 for a host-only plan */
  int n_colours;              /* colour classes (coloured scatter) or 0 */
  int64_t lattice[3];         /* L_a = k n_a + 1 (1 for unused axes) */
  int64_t n_lattice;          /* vector length expected by apply / vjp */
  int64_t n_cells, n_active_cells, n_cut_cells;
  int64_t n_active_dofs;      /* nodes of active cells */
  int64_t n_support_dofs;     /* distinct nodes touched by the face patches */
  int64_t n_faces[3];         /* ghost faces per normal axis */
  int64_t n_faces_total;
  int64_t n_patch_dofs;       /* (2k+1)(k+1)^(d-1) nodes per face patch */
  int64_t n_batches;          /* workgroups of one face-parallel launch */
  int64_t n_boxes;            /* box scatter: bricks with faces (workgroups of one launch) */
  int64_t n_visits;           /* box scatter: face visits (faces split between bricks count twice) */
  int64_t n_halo_slots;       /* box scatter: halo slots (values passed between the two kernels) */
  int64_t n_halo_nodes;       /* box scatter: support nodes on shared box faces */
  int brick;                  /* box scatter: brick edge in cells */
  double flops_per_face;      /* arithmetic of one face in the kernel, 2 per FMA (with the order
                                 coupling for GHOST_MACRO_PATCH) */
  double bytes_fp64;          /* compulsory bytes of an accumulating FP64 apply: 24 per support DoF */
  double bytes_fp32;          /* same for FP32: 12 per support DoF */
  int64_t n_inside_dofs;      /* nodes of inside cells (the interior Laplacian's nodes) */
  int n_gamma;                /* coefficients of the penalty: k, or 1 with GHOST_MACRO_PATCH */
  int macro;                  /* 1 for a GHOST_MACRO_PATCH context */
  int64_t n_cell_chunks;      /* chunks of the interior Laplacian (see ghost_cell_chunks) */
} ghost_stats;

/*
 * Build a context: classify cells, collect the ghost faces (§2.2, Fig. 1), order
 * them for locality (and colour them if GHOST_COLOURED), compute the 1D tables
 * (jump vectors of the two-cell patch and the reference mass matrix, §2.4) in
 * extended precision, and upload everything to `device`.
 *   k       polynomial degree, 1..GHOST_KMAX
 *   gamma   HOST array of k coefficients gamma_1..gamma_k, finite and >= 0 (one, gamma_M, with
 *           GHOST_MACRO_PATCH)
 *   device  HIP device ordinal, or -1 for a host-only plan (no GPU touched; only
 *           ghost_info / ghost_faces / ghost_tables / ghost_destroy are valid on it)
 *   out     receives the new context (owned by the caller; free with ghost_destroy)
 * Errors: GHOST_EINVAL (null pointer, dim not 2/3, n < 2, h <= 0, k out of range,
 * bad gamma, bad level set, lattice above 2^31 nodes per axis plane, unknown flags,
 * GHOST_MACRO_PATCH with a face-parallel scatter), GHOST_ENOMEM,
 * GHOST_EHIP.  On error nothing is leaked and *out is left NULL.
 */
int ghost_setup(const ghost_mesh *mesh, const ghost_levelset *ls, int k, const double *gamma,
                unsigned flags, int device, ghost_ctx **out);

/*
 * Replace gamma (G is linear in gamma, §2.4 summed-penalty equation).  Stream-ordered:
 * applies enqueued later on `stream` see the new values.
 *   gamma_on_device = 0: HOST array of n_gamma doubles (k, or 1 with GHOST_MACRO_PATCH),
 *                        validated (finite, >= 0).
 *   gamma_on_device = 1: DEVICE array of n_gamma doubles, read by a kernel on `stream`;
 *                        not validated.
 */
int ghost_set_gamma(ghost_ctx *ctx, const double *gamma, int gamma_on_device, void *stream);

/*
 * y (+)= G u in FP64 (Algorithm 1, face loop: gather, local apply, scatter).
 *   u, y        DEVICE arrays of n_lattice doubles; must not overlap.
 *   accumulate  1: y += G u.  0: y = G u on the support (y outside the support is
 *               left untouched: pass a zeroed y once to get G u everywhere).
 * With atomic scatter the summation order, hence the last bits, may vary run to run.
 */
int ghost_apply(ghost_ctx *ctx, const double *u, double *y, int accumulate, void *stream);

/* Same in FP32: FP32 input, output, tables (h-powers folded in FP64 first) and accumulation. */
int ghost_apply_f32(ghost_ctx *ctx, const float *u, float *y, int accumulate, void *stream);

/*
 * Pull-back of a cotangent w on y = G(gamma) u (G symmetric, linear in gamma):
 *   du (+)= G w            (DEVICE, n_lattice doubles; accumulate_du as in ghost_apply)
 *   dgamma[j] = w^T G_j u  (DEVICE, n_gamma doubles, overwritten), G_j = dG/dgamma_j
 *                          (with GHOST_MACRO_PATCH: one value, w^T S u / gamma_M evaluated as such).
 * dgamma is reduced deterministically (fixed order, no atomics).  u, w, du must not
 * overlap du.
 */
int ghost_vjp(ghost_ctx *ctx, const double *u, const double *w, double *du, double *dgamma,
              int accumulate_du, void *stream);

/*
 * Diagonal lumped mass of the active cells on the lattice, written to `diag`
 * (DEVICE, n_lattice doubles, fully overwritten):
 *   M_ii = sum over active cells K containing node i of h^d prod_a w_{i_a},
 * with w the GLL quadrature weights on [0, 1].  Zero on inactive nodes.
 */
int ghost_mass_diag(ghost_ctx *ctx, double *diag, void *stream);

/*
 * diag (+)= the diagonal of G (§2.4: for a patch node at normal position i and tangential
 * positions t, sum_j gamma_j h^{d-1-2j} g_j[i]^2 times the diagonal mass entries), summed over
 * the faces, for the current gamma; with GHOST_MACRO_PATCH, gamma_M h^{d-2} sum_ab H_ab g_a[i] g_b[i]
 * with the order coupling H.  diag: DEVICE array of n_lattice doubles; accumulate = 0 zeroes
 * the support first (other entries untouched).  Stream-ordered; uses FP64 atomics (meant for
 * preconditioner set-up, not for the hot loop).
 */
int ghost_diag(ghost_ctx *ctx, double *diag, int accumulate, void *stream);

/*
 * Interior-cell Laplacian (the cell term of the weak form, §2.1, on the cells the boundary does not cut,
 * evaluated by sum factorisation as in §2.5 and Algorithm 1):
 *   y += sum over INSIDE cells K of K_K u_K,  [K_K]_ab = integral_K grad phi_a . grad phi_b,
 * so that ghost_cell_apply followed by ghost_apply (accumulate = 1) gives (K_inside + G) u, the
 * operator of the paper's vmult without its cut-cell part.  u, y: DEVICE arrays of n_lattice values
 * (u != y); y is only added to (pass a zeroed y for K_inside u).  Stream-ordered; one launch per colour
 * of the chunks of consecutive inside cells along x (chunks of a colour share no node), no atomics.
 */
int ghost_cell_apply(ghost_ctx *ctx, const double *u, double *y, void *stream);
int ghost_cell_apply_f32(ghost_ctx *ctx, const float *u, float *y, void *stream);

/*
 * Single-face microbenchmark (the computational-efficiency experiment of §3, ghost-penalty column):
 * for n_faces independent faces, out = reps * G_F in, each face's operator applied `reps` times to the
 * same values by the apply's per-face pipeline (normal contraction, tangential masses, expansion),
 * without the gather from the lattice and the scatter, so the run is compute-bound.  G_F is the face
 * operator of the context's d, k, h and gamma in the face's local coordinates (the same for every
 * normal axis).  in, out: DEVICE arrays of n_faces * (2k+1) * (k+1)^(d-1) values in the layout
 * [face][normal node i = 0..2k][tangential line t], t = t1 + (k+1) t2 with t1, t2 along the tangential
 * axes in increasing order; out is overwritten.  n_faces >= 0, reps >= 1.  Stream-ordered.
 * GHOST_ESTATE for a GHOST_MACRO_PATCH context (derivative-jump form only).
 */
int ghost_face_bench(ghost_ctx *ctx, const double *in, double *out, int64_t n_faces, int reps, void *stream);
int ghost_face_bench_f32(ghost_ctx *ctx, const float *in, float *out, int64_t n_faces, int reps, void *stream);

/* Conjugate gradients on (M + G) x = b over the active nodes (M as in ghost_mass_diag). */
#define GHOST_CG_FP64 0  /* plain FP64 CG */
#define GHOST_CG_MIXED 1 /* FP64 outer refinement of the true residual, FP32 inner CG */

typedef struct {
  int mode;          /* GHOST_CG_FP64 or GHOST_CG_MIXED */
  double tol;        /* stop when |b - A x|_2 <= tol |b|_2 (true residual, FP64) */
  int max_iter;      /* cap on the total number of (inner) iterations */
  double inner_tol;  /* mixed: relative residual reduction of each inner solve */
  int check_every;   /* recompute the true residual every this many iterations (FP64 mode, and
                        every FP64 / Jacobi-preconditioned stopping test) */
  int precond;       /* GHOST_CG_NONE or GHOST_CG_JACOBI */
} ghost_cg_opts;
#define GHOST_CG_NONE 0   /* unpreconditioned */
#define GHOST_CG_JACOBI 1 /* diagonal of M + G (computed on the device for the current gamma) */

typedef struct {
  int iterations;          /* total (inner) iterations */
  int outer;               /* outer refinement steps (mixed), else 1 */
  int converged;           /* 1 if tol was reached */
  double rel_residual;     /* final true relative residual |b - A x| / |b| (FP64) */
} ghost_cg_result;

/*
 * Solve (M + G) x = b from x = 0.  b, x: DEVICE arrays of n_lattice doubles; b must be
 * zero on inactive nodes.  x is written on the active nodes only; its other entries are
 * left as they were.  Synchronous: returns when the solve ends.  Allocates its workspace
 * on the first call (kept until ghost_destroy).  The host reads the recursive residual of the
 * unpreconditioned and the inner FP32 iterations every 8 iterations, so a solve may run up to 7
 * iterations past the point where it would have stopped.
 */
int ghost_cg(ghost_ctx *ctx, const double *b, double *x, const ghost_cg_opts *opts,
             ghost_cg_result *res, void *stream);

/* Sizes and counts of the context (host struct filled by the call). */
int ghost_info(const ghost_ctx *ctx, ghost_stats *out);

/*
 * Copy the ghost faces normal to `axis` to the HOST array `out` as 4 int32 per face:
 * lower-cell multi-index c0, c1, c2 (c2 = 0 in 2D) and colour (-1 without colouring),
 * in the library's internal order.  `cap` is the capacity of `out` in faces; fails with
 * GHOST_EINVAL if it is smaller than n_faces[axis].
 */
int ghost_faces(const ghost_ctx *ctx, int axis, int32_t *out, int64_t cap);

/*
 * Copy the 1D tables to HOST arrays (any may be NULL):
 *   jumps  k x (2k+1): row j-1 = jumps of the j-th derivative of the 2k+1 two-cell
 *          reference patch functions across the face, right minus left (§2.4, G^1_j = g g^T)
 *   mass   (k+1) x (k+1): exact reference mass matrix M^1 on [0, 1] (§2.4)
 *   nodes, weights  k+1 GLL nodes and weights on [0, 1]
 */
int ghost_tables(const ghost_ctx *ctx, double *jumps, double *mass, double *nodes, double *weights);

/*
 * Copy the box-scatter layout to HOST arrays (inspection and tests); each may be NULL to skip it.
 *   boxes   7 int32 per brick: node origin[3], first visit, visit count, first run, run count
 *                                                                         (capacity box_cap boxes)
 *   visits  packed faces: c0 | c1 << 20 | c2 << 40 | axis << 60 | half << 62, half 0 = whole patch,
 *           1 = lower cell only (patch planes 0..k), 2 = upper cell only (planes k+1..2k)  (visit_cap)
 *   runs    4 int64 per run of box nodes: lattice start, accumulator index, length, halo slot
 *           (-1 = written to y)                                           (capacity run_cap runs)
 * GHOST_EINVAL if a capacity is too small.
 */
/*
 * Copy the chunks of the interior Laplacian (ghost_cell_apply) to the HOST array `out` (inspection and
 * tests), 3 int64 per chunk: lattice index of the first node of its first cell, the number of
 * consecutive inside cells along x it holds, and its colour (the launch it runs in; chunks of one
 * colour share no node).  `cap` is the capacity in chunks; GHOST_EINVAL if it is below n_cell_chunks.
 */
int ghost_cell_chunks(const ghost_ctx *ctx, int64_t *out, int64_t cap);

int ghost_box_layout(const ghost_ctx *ctx, int32_t *boxes, int64_t box_cap, uint64_t *visits,
                     int64_t visit_cap, int64_t *runs, int64_t run_cap);

/*
 * Per-kernel timing (a profiling aid).  ghost_set_timing(ctx, 1) makes every later apply, FP32
 * apply and VJP on the context record HIP events on its stream around its scatter kernel
 * (the box kernel, or all face kernels) and around the halo pass that follows it;
 * ghost_set_timing(ctx, 0) stops recording.  ghost_kernel_times waits for the recorded
 * events, returns the summed durations in milliseconds (main_ms: scatter kernels, halo_ms:
 * halo pass) and the number of recorded calls in *calls, and starts a new sum.  Event
 * records are not meant for streams under graph capture.  Host pointers; NULL outputs are
 * skipped.  GHOST_ESTATE on a host-only context.
 */
int ghost_set_timing(ghost_ctx *ctx, int on);
int ghost_kernel_times(ghost_ctx *ctx, double *main_ms, double *halo_ms, int64_t *calls);

/* Release the context and every allocation it owns.  NULL is a no-op. */
void ghost_destroy(ghost_ctx *ctx);

/* Message of the last failing call on this thread ("" if none). */
const char *ghost_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GHOST_H */
