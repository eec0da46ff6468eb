"""CPU tests of libghost's host side: exports, plan vs the oracle, colouring, error paths.

No GPU is touched: contexts are built with device = -1 (host-only plans).
"""

import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import mesh as omesh, patch as opatch
from oracle.basis import gll_nodes, gll_weights
from oracle.operator import GhostOracle
from paper_2503_00246_amd import _lib as L
from paper_2503_00246_amd.operator import GhostOperator
from paper_2503_00246_amd.workloads import WORKLOADS, gamma_paper

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_exports_every_declared_symbol(lib):
    with open(os.path.join(ROOT, "include", "ghost.h")) as f:
        text = f.read()
    declared = set(re.findall(r"^\s*(?:int|void|const char \*)\s*(ghost_\w+)\s*\(", text, re.M))
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name)


def _workload(name):
    """A named workload, or a multiple-ball one named balls3d_q<k>_<n>_b<balls>."""
    if name in WORKLOADS:
        return WORKLOADS[name]
    from paper_2503_00246_amd.workloads import multiball_workload
    _, q, n, b = name.split("_")
    return multiball_workload(int(q[1:]), int(n), int(b[1:]))


def _host(w, scatter="box", **kw):
    return GhostOperator.from_workload(w, scatter=scatter, device=-1, **kw)


@pytest.mark.parametrize("k", range(1, 8))
def test_tables_match_oracle(k):
    w = WORKLOADS["disk2d_q2_32"]
    op = GhostOperator(2, w.n, w.lo, w.h, k, gamma_paper(k, w.h), centre=w.centre, radius=w.radius, device=-1)
    t = op.tables()
    J = opatch.jump_vectors_reference(k)
    jumps = np.array([[float(v) for v in J[j]] for j in range(1, k + 1)])
    mass = np.array([[float(v) for v in r] for r in opatch.mass_reference(k)])
    np.testing.assert_allclose(t["jumps"], jumps, rtol=0, atol=2e-16 * np.abs(jumps).max())
    np.testing.assert_allclose(t["mass"], mass, rtol=0, atol=2e-16)
    np.testing.assert_allclose(t["nodes"], [float(x) for x in gll_nodes(k)], rtol=0, atol=2e-16)
    np.testing.assert_allclose(t["weights"], [float(x) for x in gll_weights(k)], rtol=0, atol=2e-16)


@pytest.mark.parametrize("k", range(1, 8))
def test_tables_reflection_symmetry_exact(k):
    """Reflection about the face maps patch node i to 2k-i; the jump of the order-m derivative changes by
    (-1)^(m+1) and the mass matrix is centro-symmetric.  The box kernel folds its contractions with these
    identities, so the tables must satisfy them bit for bit (the oracle's vectors do up to rounding)."""
    w = WORKLOADS["disk2d_q2_32"]
    op = GhostOperator(2, w.n, w.lo, w.h, k, gamma_paper(k, w.h), centre=w.centre, radius=w.radius, device=-1)
    t = op.tables()
    J = np.asarray(t["jumps"])
    for m in range(1, k + 1):
        assert np.array_equal(J[m - 1][::-1], (-1) ** (m + 1) * J[m - 1])
    M = np.asarray(t["mass"])
    assert np.array_equal(M, M.T) and np.array_equal(M, M[::-1, ::-1])
    J_or = opatch.jump_vectors_reference(k)
    for m in range(1, k + 1):  # the oracle's (independent) vectors obey the same identity to rounding
        v = np.array([float(x) for x in J_or[m]])
        np.testing.assert_allclose(v[::-1], (-1) ** (m + 1) * v, rtol=0, atol=1e-13 * np.abs(v).max())


def test_generated_tables_match_runtime_tables():
    """The kernels' compile-time jump vectors and mass matrices (written at build time) are bit-identical
    to the tables the library builds at run time (and which the oracle comparison above pins)."""
    path = os.path.join(ROOT, "_build", "ghost_tables_gen.h")
    text = open(path).read()
    blocks = re.findall(r"struct Tab1d<(\d+)> \{\s*static constexpr double g\[\d+\] = \{([^}]*)\};\s*"
                        r"static constexpr double M\[\d+\] = \{([^}]*)\};", text)
    assert [int(b[0]) for b in blocks] == list(range(2, 9))
    w = WORKLOADS["disk2d_q2_32"]
    for K, g, M in blocks:
        k = int(K) - 1
        op = GhostOperator(2, w.n, w.lo, w.h, k, gamma_paper(k, w.h), centre=w.centre, radius=w.radius, device=-1)
        t = op.tables()
        gv = np.array([float.fromhex(x.strip()) for x in g.split(",")])
        Mv = np.array([float.fromhex(x.strip()) for x in M.split(",")])
        assert np.array_equal(gv, np.asarray(t["jumps"]).ravel())
        assert np.array_equal(Mv, np.asarray(t["mass"]).ravel())


@pytest.mark.parametrize("name", ["disk2d_q2_32", "ball3d_q3_64", "balls3d_q3_32_b8", "balls3d_q2_24_b16"])
def test_plan_matches_oracle(name):
    w = _workload(name)
    op = _host(w)
    cls = (omesh.classify_balls(w.n, w.lo, w.h, w.balls) if w.balls
           else omesh.classify_ball(w.n, w.lo, w.h, w.centre, w.radius))
    faces = omesh.ghost_faces(cls)
    st = op.stats
    assert st["n_active_cells"] == int(np.sum(cls != 0))
    assert st["n_cut_cells"] == int(np.sum(cls == 2))
    for a in range(w.d):
        got = op.faces(a)[:, :w.d]
        np.testing.assert_array_equal(got, faces[a])
        assert st["n_faces"][a] == len(faces[a])
    assert st["n_patch_dofs"] == w.n_p
    assert st["n_lattice"] == w.n_lattice
    # support = union of the patches, active = nodes of active cells
    L_ = w.lattice
    sup = np.unique(np.concatenate([omesh.patch_dofs(faces[a], w.k, a, L_).ravel() for a in range(w.d)]))
    assert st["n_support_dofs"] == len(sup)
    assert st["bytes_fp64"] == 24 * len(sup)
    from oracle.cell import cell_dofs
    inside = np.argwhere(cls == omesh.INSIDE)
    assert st["n_inside_dofs"] == (len(np.unique(cell_dofs(inside, w.k, w.lattice))) if len(inside) else 0)
    if w.d == 2:
        o = GhostOracle(w.d, w.n, w.lo, w.h, w.k, w.gamma(), centre=w.centre, radius=w.radius)
        assert st["n_active_dofs"] == int(np.sum(o.lumped_mass() > 0))


def test_flop_count_formula():
    """Rank-k cost per face: 2k(2k+1)(k+1)^{d-1} + (d-1)k(k+1)^d FMAs (2 flops each)."""
    for name in ["disk2d_q2_32", "ball3d_q3_64"]:
        w = WORKLOADS[name]
        k, d = w.k, w.d
        fma = 2 * k * (2 * k + 1) * (k + 1) ** (d - 1) + (d - 1) * k * (k + 1) ** d
        assert _host(w).stats["flops_per_face"] == 2 * fma
        # the macro-patch form adds the order coupling: entries (i, j) with i + j even, per line
        pairs = sum(1 for i in range(k) for j in range(k) if (i + j) % 2 == 0)
        macro = GhostOperator.from_workload(w, device=-1, penalty="macro")
        assert macro.stats["flops_per_face"] == 2 * (fma + pairs * (k + 1) ** (d - 1))


@pytest.mark.parametrize("name", ["disk2d_q2_32", "ball3d_q3_64"])
def test_colouring_is_race_free(name):
    """No two faces of one colour share a lattice node (exact check with the oracle's patch numbering)."""
    w = WORKLOADS[name]
    op = _host(w, scatter="coloured")
    per_axis = 3 * 2 ** (w.d - 1)
    assert op.stats["n_colours"] == w.d * per_axis
    owner = {}
    for a in range(w.d):
        f = op.faces(a)
        dofs = omesh.patch_dofs(f[:, :w.d].astype(np.int64), w.k, a, w.lattice)
        for col in np.unique(f[:, 3]):
            sel = f[:, 3] == col
            flat = dofs[sel].ravel()
            assert len(np.unique(flat)) == len(flat), f"colour {col} has a shared node"
            owner[col] = owner.get(col, 0) + sel.sum()
    assert sum(owner.values()) == op.stats["n_faces_total"]


def test_cell_class_level_set_matches_ball():
    w = WORKLOADS["disk2d_q2_32"]
    cls = omesh.classify_ball(w.n, w.lo, w.h, w.centre, w.radius)
    flat = cls.ravel(order="F")  # x fastest
    a = _host(w)
    b = GhostOperator(2, w.n, w.lo, w.h, w.k, w.gamma(), cell_class=flat, device=-1)
    for ax in range(2):
        np.testing.assert_array_equal(a.faces(ax), b.faces(ax))
    assert a.stats["n_support_dofs"] == b.stats["n_support_dofs"]


def test_empty_face_set_is_valid():
    """A ball strictly inside one cell's neighbourhood without ghost faces: zero faces, valid plan."""
    op = GhostOperator(2, (8, 8), (-1, -1), 0.25, 2, [1.0, 1.0], centre=(5.0, 5.0), radius=0.1, device=-1)
    assert op.stats["n_faces_total"] == 0 and op.stats["n_support_dofs"] == 0


def _raw_setup(lib, dim=2, n=(8, 8, 8), h=0.25, k=2, gamma=(1.0, 1.0), kind=0, radius=0.5, flags=0, device=-1,
               cls=None, null=None):
    m = L.GhostMesh()
    m.dim = dim
    for a in range(3):
        m.n[a] = n[a]
        m.lo[a] = -1.0
    m.h = h
    ls = L.GhostLevelset()
    ls.kind = kind
    ls.radius = radius
    if cls is not None:
        ls.cell_class = cls
    g = (ctypes.c_double * max(1, len(gamma)))(*gamma)
    out = ctypes.c_void_p()
    args = [ctypes.byref(m), ctypes.byref(ls), k, g, flags, device, ctypes.byref(out)]
    if null is not None:
        args[null] = None
    rc = lib.ghost_setup(*args)
    if rc == 0:
        lib.ghost_destroy(out)
    return rc, lib.ghost_last_error().decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(dim=4), "dim"), (dict(k=0), "k must"), (dict(k=8, gamma=(1.0,) * 8), "k must"),
    (dict(n=(1, 8, 8)), "n[0]"), (dict(h=0.0), "h must"), (dict(h=float("nan")), "h must"),
    (dict(gamma=(1.0, -1.0)), "gamma"), (dict(gamma=(1.0, float("inf"))), "gamma"),
    (dict(radius=-1.0), "radius"), (dict(kind=7), "kind"), (dict(kind=1), "cell_class"),
    (dict(flags=64), "flags"), (dict(device=-2), "device"), (dict(null=0), "null"), (dict(null=3), "null"),
    (dict(null=6), "out"),
])
def test_setup_rejects_bad_arguments(lib, kw, needle):
    rc, msg = _raw_setup(lib, **kw)
    assert rc == L.GHOST_EINVAL and needle in msg, msg


@pytest.mark.parametrize("balls,needle", [
    ([], "n_balls"), ([(0.0, 0.0, 0.0, -0.5)], "radius"), ([(0.0, 0.0, 0.0, 0.5), (float("nan"), 0.0, 0.0, 0.5)], "centre"),
    ([(0.0, 0.0, 0.0, float("inf"))], "radius"),
])
def test_setup_rejects_bad_balls(balls, needle):
    from paper_2503_00246_amd._lib import GhostError
    with pytest.raises(GhostError, match=needle):
        GhostOperator(3, (8, 8, 8), (-1, -1, -1), 0.25, 2, [1.0, 1.0], balls=np.array(balls, dtype=np.float64).reshape(-1, 4),
                      device=-1)


@pytest.mark.parametrize("kw,needle", [
    (dict(flags=L.GHOST_MACRO_PATCH | L.GHOST_ATOMIC, gamma=(1.0,)), "box scatter"),
    (dict(flags=L.GHOST_MACRO_PATCH | L.GHOST_COLOURED, gamma=(1.0,)), "box scatter"),
    (dict(flags=L.GHOST_MACRO_PATCH, gamma=(-1.0,)), "gamma"),
    (dict(flags=L.GHOST_MACRO_PATCH, gamma=(float("nan"),)), "gamma"),
])
def test_macro_setup_rejections(lib, kw, needle):
    rc, msg = _raw_setup(lib, **kw)
    assert rc == L.GHOST_EINVAL and needle in msg, msg


def test_macro_context_stats():
    w = WORKLOADS["disk2d_q2_32"]
    m = GhostOperator.from_workload(w, device=-1, penalty="macro")
    assert m.stats["macro"] == 1 and m.stats["n_gamma"] == 1 and m.n_gamma == 1
    g = GhostOperator.from_workload(w, device=-1)
    assert g.stats["macro"] == 0 and g.stats["n_gamma"] == w.k
    for key in ("n_faces_total", "n_support_dofs", "n_boxes"):
        assert m.stats[key] == g.stats[key]
    with pytest.raises(ValueError):
        GhostOperator.from_workload(w, device=-1, penalty="macro", gamma=[1.0, 1.0])
    with pytest.raises(ValueError):
        GhostOperator.from_workload(w, device=-1, penalty="jump")


def test_generated_macro_coupling_reproduces_oracle():
    """The kernels' compile-time order coupling H with the library's jump vectors g gives g^T H g, which
    must equal the oracle's 1D macro-patch matrix on the reference patch (assembled from the extension
    differences by quadrature, without derivatives): a check of the Taylor-coefficient derivation."""
    from oracle.macro import macro_matrix_1d
    text = open(os.path.join(ROOT, "_build", "ghost_tables_gen.h")).read()
    blocks = dict(re.findall(r"struct Tab1d<(\d+)> \{[^}]*\};[^}]*\};[^}]*\};\s*"
                             r"static constexpr double H\[\d+\] = \{([^}]*)\};", text))
    assert sorted(int(K) for K in blocks) == list(range(2, 9))
    w = WORKLOADS["disk2d_q2_32"]
    for K, H in blocks.items():
        k = int(K) - 1
        op = GhostOperator(2, w.n, w.lo, w.h, k, gamma_paper(k, w.h), centre=w.centre, radius=w.radius, device=-1)
        g = np.asarray(op.tables()["jumps"]).reshape(k, 2 * k + 1)
        Hm = np.array([float.fromhex(x.strip()) for x in H.split(",")]).reshape(k, k)
        ref = macro_matrix_1d(k, 0.0, 1.0)
        assert np.max(np.abs(g.T @ Hm @ g - ref)) <= 1e-12 * np.max(np.abs(ref)), k


@pytest.mark.parametrize("d,k,n", [(2, 2, 24), (3, 1, 14), (3, 3, 14), (3, 5, 12), (3, 7, 40), (2, 7, 200)])
def test_cell_chunks_cover_inside_cells_and_colours_share_no_node(d, k, n):
    """The interior Laplacian's chunks (runs of inside cells along x, one launch per colour): every inside
    cell of the oracle's classification lies in exactly one chunk, and no lattice node belongs to cells of
    two different chunks of one colour (so a launch needs no atomics).  The last two meshes have runs of
    inside cells longer than a chunk (16 cells at 3D k = 7, 128 at 2D k = 7), so that neighbouring chunks
    of one run are checked too."""
    centre = (0.011, 0.017, 0.023)[:d]
    h = 2.0 / n
    op = GhostOperator(d, (n,) * d, (-1.0,) * d, h, k, gamma_paper(k, h), centre=centre, radius=0.73, device=-1)
    cls = omesh.classify_ball((n,) * d, (-1.0,) * d, h, centre, 0.73)
    L = np.array([k * n + 1] * d, dtype=np.int64)
    stride = np.cumprod(np.concatenate([[1], L[:-1]]))
    chunks = op.cell_chunks()
    assert len(chunks) == op.stats["n_cell_chunks"] > 0
    first = (chunks[:, :1] // stride[None, :]) % L[None, :]          # first node multi-index per chunk
    assert np.all(first % k == 0)
    # every cell of every chunk, with its chunk id and colour
    cid = np.repeat(np.arange(len(chunks)), chunks[:, 1])
    step = np.arange(len(cid)) - np.repeat(np.cumsum(chunks[:, 1]) - chunks[:, 1], chunks[:, 1])
    cells = first[cid] // k
    cells[:, 0] += step
    covered = np.zeros(cls.shape, dtype=np.int64)
    np.add.at(covered, tuple(cells.T), 1)
    assert np.array_equal(covered, (cls == omesh.INSIDE).astype(np.int64))
    longest = max(int(c) for c in chunks[:, 1])
    if n >= 40:
        # some run is cut into several chunks
        assert (cls == omesh.INSIDE).sum(axis=0).max() > longest
    # nodes of each cell; within a colour, a node may belong to one chunk only
    loc = np.stack(np.meshgrid(*[np.arange(k + 1)] * d, indexing="ij"), -1).reshape(-1, d)
    nodes = ((k * cells[:, None, :] + loc[None, :, :]) * stride[None, None, :]).sum(-1)
    col = np.repeat(chunks[cid, 2][:, None], len(loc), axis=1).ravel()
    own = np.repeat(cid[:, None], len(loc), axis=1).ravel()
    nodes = nodes.ravel()
    order = np.lexsort((own, nodes, col))
    col, nodes, own = col[order], nodes[order], own[order]
    same = (col[1:] == col[:-1]) & (nodes[1:] == nodes[:-1])
    assert not np.any(same & (own[1:] != own[:-1]))


def test_cell_chunks_capacity_checked(lib):
    w = WORKLOADS["disk2d_q2_32"]
    op = GhostOperator.from_workload(w, device=-1)
    n = op.stats["n_cell_chunks"]
    out = np.zeros((n, 3), dtype=np.int64)
    rc = lib.ghost_cell_chunks(op._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n - 1)
    assert rc == L.GHOST_EINVAL and "capacity" in lib.ghost_last_error().decode()
    assert lib.ghost_cell_chunks(op._h, None, n) == L.GHOST_EINVAL


def test_bad_cell_class_value(lib):
    cls = (ctypes.c_byte * 64)(*([0] * 63 + [5]))
    rc, msg = _raw_setup(lib, kind=1, cls=ctypes.cast(cls, ctypes.POINTER(ctypes.c_byte)))
    assert rc == L.GHOST_EINVAL and "cell_class" in msg


def test_host_only_context_refuses_device_work(lib):
    w = WORKLOADS["disk2d_q2_32"]
    op = _host(w)
    p = ctypes.c_void_p(16)
    q = ctypes.c_void_p(1 << 40)
    assert lib.ghost_apply(op._h, p, q, 0, None) == L.GHOST_ESTATE
    assert lib.ghost_apply_f32(op._h, p, q, 0, None) == L.GHOST_ESTATE
    assert lib.ghost_vjp(op._h, p, p, q, q, 0, None) == L.GHOST_ESTATE
    assert lib.ghost_mass_diag(op._h, p, None) == L.GHOST_ESTATE
    assert lib.ghost_set_gamma(op._h, p, 0, None) == L.GHOST_ESTATE
    assert lib.ghost_diag(op._h, p, 0, None) == L.GHOST_ESTATE
    assert lib.ghost_set_timing(op._h, 1) == L.GHOST_ESTATE
    assert lib.ghost_kernel_times(op._h, None, None, None) == L.GHOST_ESTATE
    assert lib.ghost_set_timing(None, 1) == L.GHOST_EINVAL
    assert lib.ghost_apply(None, p, q, 0, None) == L.GHOST_EINVAL
    assert lib.ghost_info(None, None) == L.GHOST_EINVAL
    small = np.zeros((1, 4), dtype=np.int32)
    assert lib.ghost_faces(op._h, 0, small.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 1) == L.GHOST_EINVAL
    assert lib.ghost_faces(op._h, 5, small.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 1) == L.GHOST_EINVAL
    lib.ghost_destroy(None)  # no-op


@pytest.mark.parametrize("name", ["disk2d_q2_32", "ball3d_q3_64", "small3d_q5_24", "small3d_q7_14", "small3d_q2_24",
                                  "small3d_q1_20"])
def test_box_layout(name):
    """Box scatter layout: runs of all boxes cover the support exactly; every support node is written to y
    by exactly one box, the first (in box order) that touches it, and routed through a halo slot by every
    later box touching it; each face is visited once (whole patch) or twice (lower / upper cell, by the
    bricks of those cells); run accumulator indices are the box-relative node coordinates,
    x + P*(y + E*z) with E the accumulator extent, P = E + 1."""
    from paper_2503_00246_amd.workloads import Workload
    extra = {"small3d_q5_24": Workload("s", 3, 5, (24,) * 3, (-1.0,) * 3, (0.011, 0.017, 0.023), 0.73),
             "small3d_q7_14": Workload("s", 3, 7, (14, 13, 12), (-1.0,) * 3, (0.011, 0.017, 0.023), 0.73),
             "small3d_q2_24": Workload("s", 3, 2, (24,) * 3, (-1.0,) * 3, (0.011, 0.017, 0.023), 0.73),
             "small3d_q1_20": Workload("s", 3, 1, (20, 19, 18), (-1.0,) * 3, (0.011, 0.017, 0.023), 0.73)}
    w = WORKLOADS.get(name) or extra[name]
    op = _host(w)
    boxes, visits, runs = op.box_layout()
    d, k = w.d, w.k
    B = 15 // k if d == 3 else 63 // k
    NB = k * B + 1
    E = 16 if d == 3 else 64
    P = E + 1
    assert NB <= E
    assert op.stats["brick"] == B
    L_ = np.array(list(w.lattice) + [1] * (3 - d))
    cls = omesh.classify_ball(w.n, w.lo, w.h, w.centre, w.radius)
    faces = omesh.ghost_faces(cls)
    sup = np.unique(np.concatenate([omesh.patch_dofs(faces[a], k, a, w.lattice).ravel() for a in range(d)]))
    # runs: cover the support; exclusive vs shared consistent
    box_of_run = np.repeat(np.arange(len(boxes)), boxes[:, 6])
    order = np.concatenate([np.arange(b[5], b[5] + b[6]) for b in boxes])
    runs = runs[order]
    nodes = np.concatenate([np.arange(s_, s_ + n_) for s_, _, n_, _ in runs])
    shared = np.concatenate([np.full(n_, sl >= 0) for _, _, n_, sl in runs])
    rbox = np.repeat(box_of_run, runs[:, 2])
    assert np.array_equal(np.unique(nodes), sup)
    # a box touches a node at most once; exactly one box writes each support node to y, and it is the
    # first of the boxes touching the node; the others use halo slots
    assert len(np.unique(np.stack([nodes, rbox]), axis=1)[0]) == len(nodes)
    direct = nodes[~shared]
    assert np.array_equal(np.sort(direct), sup)
    first_box = np.full(int(nodes.max()) + 1, len(boxes), dtype=np.int64)
    np.minimum.at(first_box, nodes, rbox)
    assert np.array_equal(rbox[~shared], first_box[direct])
    assert np.all(rbox[shared] > first_box[nodes[shared]])
    # at most one visit per thread of the box kernel
    assert boxes[:, 4].max() <= 512 and boxes[:, 4].min() >= 1
    assert op.stats["n_halo_slots"] == int(shared.sum())
    assert op.stats["n_halo_nodes"] == len(np.unique(nodes[shared]))
    slots = np.concatenate([np.arange(sl, sl + n_) for _, _, n_, sl in runs if sl >= 0] + [np.zeros(0, np.int64)])
    assert np.array_equal(np.sort(slots), np.arange(len(slots)))
    # accumulator index = box-relative coordinates
    I = np.stack([nodes % L_[0], (nodes // L_[0]) % L_[1], nodes // (L_[0] * L_[1])], -1)
    rel = I - boxes[rbox, 0:3]
    assert np.all(rel >= 0) and np.all(rel[:, :d] < NB)
    accs = np.concatenate([np.arange(a_, a_ + n_) for _, a_, n_, _ in runs])
    assert np.array_equal(accs, rel[:, 0] + P * (rel[:, 1] + E * rel[:, 2]))
    # visits
    v = visits.astype(np.uint64)
    c = np.stack([(v & 0xFFFFF), (v >> 20) & 0xFFFFF, (v >> 40) & 0xFFFFF], -1).astype(np.int64)
    ax = ((v >> 60) & 3).astype(np.int64)
    half = ((v >> 62) & 3).astype(np.int64)
    vbox = np.repeat(np.arange(len(boxes)), boxes[:, 4])
    vorder = np.concatenate([np.arange(b[3], b[3] + b[4]) for b in boxes])
    c, ax, half = c[vorder], ax[vorder], half[vorder]
    brick = boxes[vbox, 0:3] // (k * B)
    lower = c // B
    upper = (c + np.eye(3, dtype=np.int64)[ax]) // B
    assert np.all(np.where((half == 2)[:, None], upper, lower)[:, :d] == brick[:, :d])
    assert np.all(np.all(lower == upper, axis=1) == (half == 0))
    key = ax * (1 << 60) + c[:, 0] + (c[:, 1] << 20) + (c[:, 2] << 40)
    uk, cnt = np.unique(key, return_counts=True)
    assert len(uk) == sum(len(faces[a]) for a in range(d))
    halves = {}
    for kk, h in zip(key, half):
        halves.setdefault(int(kk), []).append(int(h))
    assert all(sorted(h) in ([0], [1, 2]) for h in halves.values())
