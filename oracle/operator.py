"""Global ghost-penalty operator from dense patch matrices.  Test infrastructure only.

* Apply (Algorithm 1, face loop; §2.7 gather/scatter): y = sum over ghost
  faces F of scatter_F(G_F gather_F(u)), with G_F from patch.patch_matrix.
* Matrices of all faces with one normal are identical on a Cartesian mesh
  (§2.2, last paragraph before §2.3).  For small meshes the oracle assembles
  every face separately in its own physical coordinates (per_face=True); for
  large ones it assembles one matrix per normal axis and checks it against a
  per-face assembly on a seeded sample of faces.
* Gradients of L = 0.5 |G(gamma) u - t|^2: dL/du = G^T (G u - t),
  dL/dgamma_j = (G u - t)^T G_j u, with G_j the operator for gamma = e_j
  (G is linear in gamma, §2.4 eq. ghostPenaltyMatrixRev).
* penalty="macro": the macro-patch stabilisation of macro.macro_patch_matrix in place of the
  derivative-jump penalty, with one coefficient gamma_M (G is linear in it, so its gradient is
  (G u - t)^T G_1 u with G_1 the operator for gamma_M = 1).
* Lumped mass for the linear-solver workload: diagonal GLL mass of the
  active cells, M_ii = sum over active cells K containing node i of
  h^d prod_a w_{i_a}.
* cg_reference: textbook conjugate gradients in float64.
"""

import numpy as np
import scipy.sparse as sp

from . import mesh
from .patch import patch_matrix
from .macro import macro_patch_matrix
from .basis import gll_weights


class GhostOracle:
    """Ghost-penalty operator on a Cartesian mesh with a ball, a union of balls, or given cell classes."""

    def __init__(self, d, n, lo, h, k, gamma, centre=None, radius=None, cell_class=None,
                 per_face=False, check_faces=8, seed=0, balls=None, penalty="derivative"):
        self.d, self.n, self.lo, self.h, self.k = d, tuple(n), tuple(lo), float(h), k
        if penalty not in ("derivative", "macro"):
            raise ValueError("penalty must be 'derivative' or 'macro'")
        self.penalty = penalty
        self.n_gamma = k if penalty == "derivative" else 1
        self.gamma = np.asarray(gamma, dtype=np.float64)
        if self.gamma.shape != (self.n_gamma,):
            raise ValueError(f"need {self.n_gamma} coefficients")
        if balls:
            self.cls = mesh.classify_balls(self.n, self.lo, self.h, balls)
        elif cell_class is None:
            self.cls = mesh.classify_ball(self.n, self.lo, self.h, centre, radius)
        else:
            self.cls = np.asarray(cell_class, dtype=np.int8).reshape(self.n, order="F")
        self.L = mesh.lattice_shape(self.n, k)
        self.n_lattice = int(np.prod(self.L))
        self.faces = mesh.ghost_faces(self.cls)
        self.per_face = per_face
        self._axis_matrix = {}
        self._face_matrices = {}
        for a in range(d):
            f = self.faces[a]
            if len(f) == 0:
                continue
            if per_face:
                self._face_matrices[a] = np.stack([self._assemble(a, c) for c in f])
            else:
                self._axis_matrix[a] = self._assemble(a, f[0])
                rng = np.random.default_rng(seed + a)
                pick = rng.choice(len(f), size=min(check_faces, len(f)), replace=False)
                ref = self._axis_matrix[a]
                scale = np.max(np.abs(ref))
                for i in pick:
                    other = self._assemble(a, f[i])
                    err = np.max(np.abs(other - ref)) / scale
                    if err > 1e-13:
                        raise AssertionError(f"patch matrices differ between faces: {err:g}")

    # ------------------------------------------------------------------ assembly
    def _assemble(self, axis, lower_cell, gamma=None):
        g = self.gamma if gamma is None else gamma
        if self.penalty == "macro":
            return macro_patch_matrix(self.d, self.k, axis, lower_cell, self.lo, self.h, g)
        return patch_matrix(self.d, self.k, axis, lower_cell, self.lo, self.h, g)

    def n_faces(self):
        return sum(len(self.faces[a]) for a in range(self.d))

    def patch_dofs(self, axis):
        return mesh.patch_dofs(self.faces[axis], self.k, axis, self.L)

    def face_matrices(self, axis):
        """(nf, n_p, n_p) if per-face, else a single (n_p, n_p) matrix for the axis."""
        if self.per_face:
            return self._face_matrices[axis]
        return self._axis_matrix[axis]

    def support(self):
        """Sorted unique lattice indices touched by any ghost-face patch."""
        parts = [self.patch_dofs(a).ravel() for a in range(self.d) if len(self.faces[a])]
        if not parts:
            return np.zeros(0, dtype=np.int64)
        return np.unique(np.concatenate(parts))

    # ------------------------------------------------------------------ apply
    def apply(self, u, face_mask=None):
        """y = G u on the full lattice (float64).  face_mask: optional dict axis -> bool mask of faces."""
        u = np.asarray(u, dtype=np.float64)
        y = np.zeros(self.n_lattice)
        for a in range(self.d):
            if len(self.faces[a]) == 0:
                continue
            idx = self.patch_dofs(a)
            sel = slice(None) if face_mask is None else face_mask[a]
            idx = idx[sel]
            U = u[idx]                                    # gather: (nf, n_p)
            if self.per_face:
                Y = np.einsum("fab,fb->fa", self._face_matrices[a][sel], U)
            else:
                Y = U @ self._axis_matrix[a].T
            np.add.at(y, idx.ravel(), Y.ravel())          # scatter-add
        return y

    def apply_at(self, u, dofs):
        """Entries of G u at the given lattice indices, summing every face whose patch touches them."""
        dofs = np.asarray(dofs, dtype=np.int64)
        mark = np.zeros(self.n_lattice, dtype=bool)
        mark[dofs] = True
        masks = {}
        for a in range(self.d):
            if len(self.faces[a]):
                masks[a] = mark[self.patch_dofs(a)].any(axis=1)
            else:
                masks[a] = np.zeros(0, dtype=bool)
        return self.apply(u, face_mask=masks)[dofs]

    # ------------------------------------------------------------------ sparse forms
    def sparse(self, gamma=None):
        """Assembled global matrix (CSR, n_lattice x n_lattice)."""
        rows, cols, vals = [], [], []
        for a in range(self.d):
            f = self.faces[a]
            if len(f) == 0:
                continue
            idx = self.patch_dofs(a)
            if gamma is None and self.per_face:
                mats = self._face_matrices[a]
            elif gamma is None:
                mats = np.broadcast_to(self._axis_matrix[a], (len(f),) + self._axis_matrix[a].shape)
            elif self.per_face:
                mats = np.stack([self._assemble(a, c, gamma) for c in f])
            else:
                m = self._assemble(a, f[0], gamma)
                mats = np.broadcast_to(m, (len(f),) + m.shape)
            n_p = idx.shape[1]
            rows.append(np.repeat(idx, n_p, axis=1).ravel())
            cols.append(np.tile(idx, (1, n_p)).ravel())
            vals.append(np.asarray(mats).reshape(len(f), -1).ravel())
        if not rows:
            return sp.csr_matrix((self.n_lattice, self.n_lattice))
        return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n_lattice, self.n_lattice)).tocsr()

    def order_matrices(self):
        """G_j = dG/dgamma_j for each coefficient (gamma = e_j)."""
        out = []
        for j in range(self.n_gamma):
            e = np.zeros(self.n_gamma)
            e[j] = 1.0
            out.append(self.sparse(gamma=e))
        return out

    def gradients(self, u, t):
        """(L, dL/du, dL/dgamma) for L = 0.5 |G u - t|^2."""
        G = self.sparse()
        r = G @ u - t
        du = G.T @ r
        dg = np.array([r @ (Gj @ u) for Gj in self.order_matrices()])
        return 0.5 * float(r @ r), du, dg

    def vjp(self, u, w):
        """(G^T w, [w^T G_j u]_j): the pull-back of a cotangent w on y = G(gamma) u."""
        G = self.sparse()
        return G.T @ w, np.array([w @ (Gj @ u) for Gj in self.order_matrices()])

    # ------------------------------------------------------------------ linear solve workload
    def lumped_mass(self):
        """Diagonal GLL mass over active cells on the lattice."""
        w = np.array([float(x) for x in gll_weights(self.k)])
        diag = np.zeros(self.L[::-1])  # indexed [I_{d-1}, ..., I_0]
        active = np.argwhere(self.cls != mesh.OUTSIDE)
        local = np.ones([self.k + 1] * self.d)
        for a in range(self.d):
            shape = [1] * self.d
            shape[self.d - 1 - a] = self.k + 1
            local = local * w.reshape(shape)
        local = local * self.h ** self.d
        for c in active:
            sl = tuple(slice(self.k * c[a], self.k * c[a] + self.k + 1) for a in reversed(range(self.d)))
            diag[sl] += local
        return diag.ravel()  # C order of [I_{d-1},...,I_0] == x-fastest linear index

    def system(self):
        """(A, active) with A = M_lumped + G restricted to active nodes (CSR) and the active index list."""
        m = self.lumped_mass()
        active = np.nonzero(m > 0)[0]
        A = (sp.diags(m) + self.sparse()).tocsr()
        return A[active][:, active].tocsr(), active


def cg_reference(A, b, tol=1e-10, max_iter=100000):
    """Plain conjugate gradients from x = 0, stopping on |b - A x| <= tol |b| (true residual).

    Returns (x, iterations, true relative residual).  Parity of x beyond its
    residual is unpinned for ill-conditioned systems.
    """
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    nb = np.sqrt(b @ b)
    it = 0
    while it < max_iter:
        if np.sqrt(rr) <= tol * nb:
            true = np.linalg.norm(b - A @ x) / nb
            if true <= tol:
                break
            r = b - A @ x
            p = r.copy()
            rr = r @ r
        q = A @ p
        alpha = rr / (p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, float(np.linalg.norm(b - A @ x) / nb)
