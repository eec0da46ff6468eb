"""Cartesian mesh, level-set classification, ghost-face set, lattice numbering.

Test infrastructure only.

* Mesh (§2): N_0 x ... x N_{d-1} square/cubic cells of side h starting at lo.
* Level set (§2): phi > 0 inside the domain.  For a ball, phi = R - |x - c|.
  A cell is treated by the paper as inside, intersected ("cut") or outside
  (§2, §2.6, Algorithm 1).  How the intersection is decided is not stated;
  here a cell is active when it meets the open ball (min distance from the
  centre < R) and inside when all of it lies in the closed ball (max
  distance <= R); cut = active and not inside.
* Ghost faces (§2.2, Fig. 1): interior faces between two cut cells or
  between a cut cell and an inside cell.
* Continuous Q_k numbering (§2.4): node multi-index I_a = k*c_a + i_a on a
  lattice of L_a = k*N_a + 1 nodes per axis, linear index with x fastest,
  i = I_0 + L_0 I_1 + L_0 L_1 I_2.
"""

import itertools

import numpy as np

OUTSIDE, INSIDE, CUT = 0, 1, 2


def cell_distances(n, lo, h, centre):
    """Squared min and max distance from the ball centre to every cell (arrays indexed [c0, c1, (c2)])."""
    d = len(n)
    dmin2 = np.zeros(tuple(n))
    dmax2 = np.zeros(tuple(n))
    for a in range(d):
        c = np.arange(n[a], dtype=np.float64)
        lo_a = lo[a] + c * h
        hi_a = lo[a] + (c + 1) * h
        below = np.maximum(lo_a - centre[a], 0.0)
        above = np.maximum(centre[a] - hi_a, 0.0)
        near = np.maximum(below, above)
        far = np.maximum(np.abs(lo_a - centre[a]), np.abs(hi_a - centre[a]))
        shape = [1] * d
        shape[a] = n[a]
        dmin2 = dmin2 + (near * near).reshape(shape)
        dmax2 = dmax2 + (far * far).reshape(shape)
    return dmin2, dmax2


def classify_ball(n, lo, h, centre, radius, min_margin=1e-12):
    """Cell classes (OUTSIDE / INSIDE / CUT) for the ball, by exact distances.

    Raises if a distance is within min_margin of R^2, where the class would
    depend on rounding.
    """
    dmin2, dmax2 = cell_distances(n, lo, h, centre)
    r2 = radius * radius
    margin = min(np.min(np.abs(dmin2 - r2)), np.min(np.abs(dmax2 - r2)))
    if margin <= min_margin:
        raise ValueError(f"cell classification tie: margin {margin:g}")
    active = dmin2 < r2
    inside = dmax2 <= r2
    cls = np.full(tuple(n), OUTSIDE, dtype=np.int8)
    cls[active] = CUT
    cls[inside] = INSIDE
    return cls


def classify_balls(n, lo, h, balls, min_margin=1e-12):
    """Cell classes for the union of balls (c0, c1, c2, r), the multiple-ball problem of §3.

    A cell is active when it meets some open ball and inside when it lies in some closed ball; an
    active cell that no single ball contains is cut, also where several balls cover it together (a
    reading: the paper classifies cells by the level set's sign pattern, which it does not spell out).
    Raises on a distance within min_margin of some r^2, as classify_ball does.
    """
    d = len(n)
    active = np.zeros(tuple(n), dtype=bool)
    inside = np.zeros(tuple(n), dtype=bool)
    for b in balls:
        dmin2, dmax2 = cell_distances(n, lo, h, tuple(b[:d]))
        r2 = b[3] * b[3]
        margin = min(np.min(np.abs(dmin2 - r2)), np.min(np.abs(dmax2 - r2)))
        if margin <= min_margin:
            raise ValueError(f"cell classification tie: margin {margin:g}")
        active |= dmin2 < r2
        inside |= dmax2 <= r2
    cls = np.full(tuple(n), OUTSIDE, dtype=np.int8)
    cls[active] = CUT
    cls[inside] = INSIDE
    return cls


def classify_ball_loop(n, lo, h, centre, radius):
    """Same classification with a plain loop over cells (brute-force check of classify_ball)."""
    d = len(n)
    cls = np.zeros(tuple(n), dtype=np.int8)
    r2 = radius * radius
    for c in itertools.product(*[range(m) for m in n]):
        dmin2 = 0.0
        dmax2 = 0.0
        for a in range(d):
            lo_a = lo[a] + c[a] * h
            hi_a = lo[a] + (c[a] + 1) * h
            if centre[a] < lo_a:
                dmin2 += (lo_a - centre[a]) ** 2
            elif centre[a] > hi_a:
                dmin2 += (centre[a] - hi_a) ** 2
            dmax2 += max(abs(lo_a - centre[a]), abs(hi_a - centre[a])) ** 2
        if dmin2 < r2:
            cls[c] = INSIDE if dmax2 <= r2 else CUT
    return cls


def ghost_faces(cls):
    """Ghost faces per normal axis: dict axis -> (nf, d) int64 array of lower-cell multi-indices.

    A face between cells c and c + e_axis is a ghost face when both cells are
    active and at least one of them is cut.  Faces are listed in lexicographic
    order of the lower cell (x fastest).
    """
    d = cls.ndim
    active = cls != OUTSIDE
    cut = cls == CUT
    out = {}
    for a in range(d):
        lo_sl = [slice(None)] * d
        hi_sl = [slice(None)] * d
        lo_sl[a] = slice(0, cls.shape[a] - 1)
        hi_sl[a] = slice(1, cls.shape[a])
        sel = active[tuple(lo_sl)] & active[tuple(hi_sl)] & (cut[tuple(lo_sl)] | cut[tuple(hi_sl)])
        # np.nonzero lists in C order of the [c0, c1, c2] array (c_last fastest);
        # sort to x-fastest lexicographic order.
        idx = np.array(np.nonzero(sel), dtype=np.int64).T.reshape(-1, d)
        key = np.zeros(len(idx), dtype=np.int64)
        for b in reversed(range(d)):
            key = key * cls.shape[b] + idx[:, b]
        out[a] = idx[np.argsort(key, kind="stable")]
    return out


def ghost_faces_loop(cls):
    """Brute-force face set: test every interior face with a plain loop."""
    d = cls.ndim
    out = {a: [] for a in range(d)}
    for c in itertools.product(*[range(m) for m in reversed(cls.shape)]):
        c = tuple(reversed(c))  # x fastest
        for a in range(d):
            if c[a] + 1 >= cls.shape[a]:
                continue
            nb = list(c)
            nb[a] += 1
            nb = tuple(nb)
            p, q = cls[c], cls[nb]
            if p != OUTSIDE and q != OUTSIDE and (p == CUT or q == CUT):
                out[a].append(c)
    return {a: np.array(v, dtype=np.int64).reshape(-1, d) for a, v in out.items()}


def lattice_shape(n, k):
    return tuple(k * m + 1 for m in n)


def lattice_size(n, k):
    return int(np.prod(lattice_shape(n, k)))


def linear_index(I, L):
    """Linear lattice index of node multi-indices I (..., d) with x fastest."""
    I = np.asarray(I, dtype=np.int64)
    out = np.zeros(I.shape[:-1], dtype=np.int64)
    stride = 1
    for a in range(I.shape[-1]):
        out = out + I[..., a] * stride
        stride *= L[a]
    return out


def patch_extent(d, k, axis):
    """Nodes per axis of the two-cell patch of a face normal to `axis`: 2k+1 along the normal, k+1 else (§2.4)."""
    return tuple(2 * k + 1 if a == axis else k + 1 for a in range(d))


def patch_local_nodes(d, k, axis):
    """Local node multi-indices of the patch in its own lexicographic order (x fastest), Fig. 2."""
    ext = patch_extent(d, k, axis)
    grids = np.meshgrid(*[np.arange(e) for e in ext], indexing="ij")
    loc = np.stack([g.ravel(order="F") for g in grids], axis=-1)
    return loc  # row p has multi-index loc[p]; p = i0 + e0*i1 + e0*e1*i2


def patch_dofs(faces, k, axis, L):
    """Global lattice indices (nf, n_p) of every face's patch, in patch-lexicographic order."""
    d = faces.shape[1]
    loc = patch_local_nodes(d, k, axis)
    I = k * faces[:, None, :] + loc[None, :, :]
    return linear_index(I, L)
