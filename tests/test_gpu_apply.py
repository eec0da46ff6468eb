"""GPU parity of ghost_apply / ghost_apply_f32 against the CPU oracle (through the C ABI).

Error measure (normwise, the apply annihilates polynomials so entrywise relative
error is meaningless): |y - y_ref|_inf / |y_ref|_inf over the compared nodes.
Bars: 1e-12 for FP64, 1e-5 for FP32.
"""

import math

import numpy as np
import pytest

from oracle.operator import GhostOracle
from paper_2503_00246_amd.workloads import (WORKLOADS, SEED_U, Workload, face_subset, gamma_paper,
                                            uniform_vector)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
_ORACLES = {}


def oracle_for(w):
    if w.name not in _ORACLES:
        _ORACLES[w.name] = GhostOracle(w.d, w.n, w.lo, w.h, w.k, w.gamma(), centre=w.centre, radius=w.radius)
    return _ORACLES[w.name]


def nerr(y, ref):
    return float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))


SCATTERS = ("box", "atomic", "coloured")


def gpu_op(w, scatter="box"):
    from paper_2503_00246_amd.operator import GhostOperator
    return GhostOperator.from_workload(w, scatter=scatter)


def small(d, k, n, name=None, centre=None, radius=0.73):
    centre = centre or ((0.011, 0.017, 0.023) if d == 3 else (0.013, 0.021))
    return Workload(name or f"small_d{d}_k{k}_n{n}", d, k, (n,) * d, (-1.0,) * d, centre, radius)


@pytest.mark.parametrize("scatter", SCATTERS)
@pytest.mark.parametrize("name", ["disk2d_q2_32", "ball3d_q3_64"])
def test_apply_fp64_full_parity(name, scatter):
    w = WORKLOADS[name]
    o = oracle_for(w)
    op = gpu_op(w, scatter)
    u = uniform_vector(w.n_lattice, SEED_U)
    ref = o.apply(u)
    ut = torch.from_numpy(u).cuda()
    y = op.apply(ut).cpu().numpy()
    sup = o.support()
    assert nerr(y[sup], ref[sup]) <= TOL64
    off = np.ones(w.n_lattice, dtype=bool)
    off[sup] = False
    assert np.all(y[off] == 0)
    # accumulate mode adds, overwrite mode resets the support only
    y2 = torch.full_like(ut, 3.0)
    op.apply(ut, y2, accumulate=True)
    y2 = y2.cpu().numpy()
    assert nerr(y2[sup] - 3.0, ref[sup]) <= TOL64 and np.all(y2[off] == 3.0)
    y3 = torch.full_like(ut, 3.0)
    op.apply(ut, y3, accumulate=False)
    y3 = y3.cpu().numpy()
    assert nerr(y3[sup], ref[sup]) <= TOL64 and np.all(y3[off] == 3.0)


@pytest.mark.parametrize("scatter", SCATTERS)
@pytest.mark.parametrize("name", ["disk2d_q2_32", "ball3d_q3_64"])
def test_apply_fp32_parity(name, scatter):
    w = WORKLOADS[name]
    o = oracle_for(w)
    op = gpu_op(w, scatter)
    u = uniform_vector(w.n_lattice, SEED_U)
    ref = o.apply(u.astype(np.float32).astype(np.float64))
    y = op.apply_f32(torch.from_numpy(u.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    sup = o.support()
    assert nerr(y[sup], ref[sup]) <= TOL32


# every template instance (d = 2, 3 and k = 1..7) on small meshes, several tiles and ragged tails
@pytest.mark.parametrize("d,k,n", [(2, k, 12) for k in range(1, 8)] + [(3, k, 10) for k in range(1, 8)])
def test_apply_all_degrees(d, k, n):
    w = small(d, k, n)
    o = GhostOracle(w.d, w.n, w.lo, w.h, w.k, w.gamma(), centre=w.centre, radius=w.radius)
    op = gpu_op(w)
    assert op.stats["n_faces_total"] == o.n_faces()
    assert op.stats["n_batches"] >= 2
    u = uniform_vector(w.n_lattice, SEED_U)
    ref = o.apply(u)
    sup = o.support()
    ut = torch.from_numpy(u).cuda()
    ref32 = o.apply(u.astype(np.float32).astype(np.float64))
    for scatter in SCATTERS:
        ops = gpu_op(w, scatter)
        y = ops.apply(ut).cpu().numpy()
        assert nerr(y[sup], ref[sup]) <= TOL64, scatter
        y32 = ops.apply_f32(ut.float()).cpu().numpy().astype(np.float64)
        assert nerr(y32[sup], ref32[sup]) <= TOL32, scatter


def _node_coords(w):
    from oracle.basis import gll_nodes
    xi = np.array([float(x) for x in gll_nodes(w.k)])
    out = []
    for a in range(w.d):
        I = np.arange(w.k * w.n[a] + 1)
        c = np.minimum(I // w.k, w.n[a] - 1)
        out.append(w.lo[a] + w.h * (c + xi[I - w.k * c]))
    return out


def test_null_space_and_symmetry_on_gpu():
    """G p = 0 for p in Q_k, <v, G u> = <G v, u> (ball3d_q3_64, FP64 and FP32)."""
    w = WORKLOADS["ball3d_q3_64"]
    op = gpu_op(w)
    coords = _node_coords(w)
    rng = np.random.default_rng(11)
    val = np.ones([len(c) for c in reversed(coords)])
    for a in range(w.d):
        shape = [1] * w.d
        shape[w.d - 1 - a] = len(coords[a])
        val = val * np.polynomial.Polynomial(rng.uniform(-1, 1, w.k + 1))(coords[a]).reshape(shape)
    p = torch.from_numpy(val.ravel()).cuda()
    r = torch.from_numpy(uniform_vector(w.n_lattice, 12) * float(p.abs().max())).cuda()
    gp, gr = op.apply(p), op.apply(r)
    assert float(gp.abs().max() / gr.abs().max()) <= 1e-11
    gp32, gr32 = op.apply_f32(p.float()), op.apply_f32(r.float())
    assert float(gp32.abs().max() / gr32.abs().max()) <= 1e-4
    u = torch.from_numpy(uniform_vector(w.n_lattice, 13)).cuda()
    v = torch.from_numpy(uniform_vector(w.n_lattice, 14)).cuda()
    a_, b_ = float(v @ op.apply(u)), float(op.apply(v) @ u)
    assert abs(a_ - b_) <= 1e-12 * abs(a_)


@pytest.mark.parametrize("scatter", SCATTERS)
def test_zero_faces_is_noop(scatter):
    from paper_2503_00246_amd.operator import GhostOperator
    op = GhostOperator(3, (8, 8, 8), (-1, -1, -1), 0.25, 3, [1.0, 1.0, 1.0], centre=(9.0, 9.0, 9.0), radius=0.5,
                       scatter=scatter)
    assert op.stats["n_faces_total"] == 0
    u = torch.ones(op.n_lattice, dtype=torch.float64, device="cuda")
    y = torch.full_like(u, 2.0)
    op.apply(u, y, accumulate=False)
    op.apply_f32(u.float(), y.float(), accumulate=True)
    du, dg = op.vjp(u, u)
    torch.cuda.synchronize()
    assert float((y - 2.0).abs().max()) == 0.0 and float(du.abs().max()) == 0.0 and float(dg.abs().max()) == 0.0


@pytest.mark.parametrize("scatter", SCATTERS)
def test_kernel_timing_records_every_call(scatter):
    """With per-kernel timing on, each apply / VJP records one event triple on the apply's stream; the
    results are the same as without it, and contexts without faces record (empty) intervals too."""
    w = WORKLOADS["ball3d_q3_64"]
    op = gpu_op(w, scatter)
    u = torch.from_numpy(uniform_vector(w.n_lattice, SEED_U)).cuda()
    ref = op.apply(u)
    op.set_timing(True)
    y = op.apply(u)
    op.apply_f32(u.float())
    op.vjp(u, u)
    op.set_timing(False)
    op.apply(u)
    t = op.kernel_times()
    assert t["calls"] == 3 and t["main_ms"] > 0 and t["halo_ms"] >= 0
    assert op.kernel_times()["calls"] == 0
    assert torch.equal(y, ref) or nerr(y.cpu().numpy(), ref.cpu().numpy()) <= TOL64
    from paper_2503_00246_amd.operator import GhostOperator
    empty = GhostOperator(3, (8, 8, 8), (-1, -1, -1), 0.25, 3, [1.0, 1.0, 1.0], centre=(9.0, 9.0, 9.0), radius=0.5,
                          scatter=scatter)
    empty.set_timing(True)
    empty.apply(torch.ones(empty.n_lattice, dtype=torch.float64, device="cuda"))
    assert empty.kernel_times()["calls"] == 1


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["ball3d_q5_128", "ball3d_q7_96"])
def test_apply_full_size_on_face_subset(name, precision):
    """Full-size meshes (128^3 Q5 and 96^3 Q7), in the benchmark's launch configuration: compare y at every
    node of a seeded 1% face sample's patches, with the oracle summing all faces touching those nodes."""
    w = WORKLOADS[name]
    op = gpu_op(w)
    o = oracle_for(w)
    faces_all = np.concatenate([np.c_[np.full(len(o.faces[a]), a), o.faces[a]] for a in range(3)])
    pick = face_subset(len(faces_all))
    dofs = []
    for a in range(3):
        sel = pick[faces_all[pick, 0] == a]
        offset = sum(len(o.faces[b]) for b in range(a))
        if len(sel):
            from oracle import mesh
            dofs.append(mesh.patch_dofs(o.faces[a][sel - offset], w.k, a, o.L).ravel())
    dofs = np.unique(np.concatenate(dofs))
    u = uniform_vector(w.n_lattice, SEED_U)
    if precision == "fp64":
        ref = o.apply_at(u, dofs)
        y = op.apply(torch.from_numpy(u).cuda())[torch.from_numpy(dofs).cuda()].cpu().numpy()
        assert nerr(y, ref) <= TOL64
    else:
        u32 = u.astype(np.float32)
        ref = o.apply_at(u32.astype(np.float64), dofs)
        y = op.apply_f32(torch.from_numpy(u32).cuda())[torch.from_numpy(dofs).cuda()].cpu().numpy()
        assert nerr(y.astype(np.float64), ref) <= TOL32


def test_apply_split_boxes():
    """k = 1 on 20 x 19 x 18 cells: bricks of 15^3 cells hold more face visits than one box, so they are
    split into several boxes over the same node box: the first of them writes their common nodes to y,
    the others add theirs through the halo pass."""
    w = Workload("split_q1", 3, 1, (20, 19, 18), (-1.0,) * 3, (0.011, 0.017, 0.023), 0.73)
    op = gpu_op(w)
    boxes, _, _ = op.box_layout()
    assert len(np.unique(boxes[:, :3], axis=0)) < len(boxes)
    o = GhostOracle(w.d, w.n, w.lo, w.h, w.k, w.gamma(), centre=w.centre, radius=w.radius)
    u = uniform_vector(w.n_lattice, SEED_U)
    ref, sup = o.apply(u), o.support()
    ut = torch.from_numpy(u).cuda()
    assert nerr(op.apply(ut).cpu().numpy()[sup], ref[sup]) <= TOL64
    y0 = torch.from_numpy(uniform_vector(w.n_lattice, SEED_U + 10)).cuda()
    ya = op.apply(ut, y0.clone(), accumulate=True).cpu().numpy()
    assert nerr(ya - y0.cpu().numpy(), ref) <= TOL64


def test_apply_graph_replay():
    """The apply allocates nothing and never waits on the host, so a stream capture of it replays: an
    FP64 overwrite and an FP32 accumulating apply captured in one HIP graph, replayed three times with
    eager work and synchronisation between the replays, each replay against the eager result (the LDS
    sums of the box kernel may add in another order, hence the normwise bars)."""
    w = WORKLOADS["ball3d_q3_64"]
    op = gpu_op(w)
    o = oracle_for(w)
    sup = torch.from_numpy(o.support()).cuda()
    u = torch.from_numpy(uniform_vector(w.n_lattice, SEED_U)).cuda()
    u32 = u.float()
    ref = op.apply(u)
    ref32 = op.apply_f32(u32).double()
    y = torch.zeros_like(u)
    y32 = torch.zeros_like(u32)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        op.apply(u, y)
        op.apply_f32(u32, y32, accumulate=True)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        op.apply(u, y, accumulate=False)
        op.apply_f32(u32, y32, accumulate=True)
    for _ in range(3):
        y.fill_(7.0)
        y32.fill_(7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got, got32 = y.cpu().numpy(), y32.double().cpu().numpy() - 7.0
        r, r32, s = ref.cpu().numpy(), ref32.cpu().numpy(), sup.cpu().numpy()
        assert nerr(got[s], r[s]) <= TOL64
        off = np.ones(w.n_lattice, dtype=bool)
        off[s] = False
        assert np.all(got[off] == 7.0)
        assert nerr(got32[s], r32[s]) <= TOL32


def _multiball(name):
    from paper_2503_00246_amd.workloads import multiball_workload
    _, q, n, b = name.split("_")
    return multiball_workload(int(q[1:]), int(n), int(b[1:]))


@pytest.mark.parametrize("name", ["balls3d_q3_32_b8", "balls3d_q5_24_b4", "balls3d_q2_40_b32", "balls3d_q7_16_b2"])
def test_multiball_parity(name):
    """The multiple-ball problem (union of seeded balls, radius inversely proportional to their number):
    FP64 and FP32 applies of every scatter against the oracle on the whole support, y untouched off it."""
    w = _multiball(name)
    o = GhostOracle(w.d, w.n, w.lo, w.h, w.k, w.gamma(), balls=w.balls)
    u = uniform_vector(w.n_lattice, SEED_U)
    ref, sup = o.apply(u), o.support()
    ref32 = o.apply(u.astype(np.float32).astype(np.float64))
    ut = torch.from_numpy(u).cuda()
    off = np.ones(w.n_lattice, dtype=bool)
    off[sup] = False
    for scatter in SCATTERS:
        op = gpu_op(w, scatter)
        assert op.stats["n_faces_total"] == o.n_faces()
        y = torch.full_like(ut, 3.0)
        op.apply(ut, y, accumulate=False)
        y = y.cpu().numpy()
        assert nerr(y[sup], ref[sup]) <= TOL64, scatter
        assert np.all(y[off] == 3.0), scatter
        y32 = op.apply_f32(ut.float()).cpu().numpy().astype(np.float64)
        assert nerr(y32[sup], ref32[sup]) <= TOL32, scatter


def test_multiball_full_size_on_face_subset():
    """128^3 Q3 with 8 balls, in the benchmark's launch configuration: y at every node of a seeded 1% face
    sample's patches, the oracle summing all faces touching those nodes."""
    w = _multiball("balls3d_q3_128_b8")
    op = gpu_op(w)
    o = GhostOracle(w.d, w.n, w.lo, w.h, w.k, w.gamma(), balls=w.balls)
    faces_all = np.concatenate([np.c_[np.full(len(o.faces[a]), a), o.faces[a]] for a in range(3)])
    pick = face_subset(len(faces_all))
    from oracle import mesh
    dofs = []
    for a in range(3):
        sel = pick[faces_all[pick, 0] == a]
        offset = sum(len(o.faces[b]) for b in range(a))
        if len(sel):
            dofs.append(mesh.patch_dofs(o.faces[a][sel - offset], w.k, a, o.L).ravel())
    dofs = np.unique(np.concatenate(dofs))
    u = uniform_vector(w.n_lattice, SEED_U)
    ref = o.apply_at(u, dofs)
    y = op.apply(torch.from_numpy(u).cuda())[torch.from_numpy(dofs).cuda()].cpu().numpy()
    assert nerr(y, ref) <= TOL64


def test_argument_errors_are_reported_before_any_launch():
    """Null and overlapping vectors are refused with GHOST_EINVAL by the C ABI (checked on the host, before
    any kernel runs); the binding refuses tensors of the wrong type, device or size."""
    import ctypes
    from paper_2503_00246_amd import _lib as L
    w = WORKLOADS["disk2d_q2_32"]
    op = gpu_op(w)
    lib = op._lib
    u = torch.zeros(w.n_lattice, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(u)
    pu, py = ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(y.data_ptr())
    shifted = ctypes.c_void_p(u.data_ptr() + 8)
    dg = torch.zeros(w.k, dtype=torch.float64, device="cuda")
    pdg = ctypes.c_void_p(dg.data_ptr())
    cases = [
        lib.ghost_apply(op._h, None, py, 0, None),
        lib.ghost_apply(op._h, pu, None, 0, None),
        lib.ghost_apply(op._h, pu, pu, 0, None),
        lib.ghost_apply(op._h, pu, shifted, 1, None),
        lib.ghost_apply_f32(op._h, pu, pu, 0, None),
        lib.ghost_cell_apply(op._h, pu, shifted, None),
        lib.ghost_vjp(op._h, pu, py, pu, pdg, 0, None),
        lib.ghost_vjp(op._h, pu, py, py, None, 0, None),
    ]
    assert all(rc == L.GHOST_EINVAL for rc in cases), cases
    torch.cuda.synchronize()
    with pytest.raises(TypeError):
        op.apply(u.float())
    with pytest.raises(ValueError):
        op.apply(u[:-1])
    with pytest.raises(ValueError):
        op.apply(u.cpu())


def test_calls_run_on_the_current_stream():
    """Inside a torch side stream (default priority) the apply, the VJP and the interior Laplacian are
    enqueued on that stream and give the default stream's results."""
    w = WORKLOADS["ball3d_q3_64"]
    op = gpu_op(w)
    u = torch.from_numpy(uniform_vector(w.n_lattice, SEED_U)).cuda()
    ref_y = op.apply(u)
    ref_du, ref_dg = op.vjp(u, ref_y)
    ref_c = op.cell_apply(u)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        y = op.apply(u)
        du, dg = op.vjp(u, y)
        c = op.cell_apply(u)
    side.synchronize()
    scale = float(ref_y.abs().max())
    assert float((y - ref_y).abs().max()) <= 1e-14 * scale
    assert float((du - ref_du).abs().max()) <= 1e-13 * float(ref_du.abs().max())
    assert float((dg - ref_dg).abs().max()) <= 1e-13 * float(ref_dg.abs().max())
    assert float((c - ref_c).abs().max()) <= 1e-14 * float(ref_c.abs().max())


def test_vjp_and_cell_graph_replay():
    """A VJP (du overwritten, dgamma reduced) and an interior-Laplacian apply captured in one HIP graph,
    replayed three times with eager resets and synchronisation between replays, each replay checked
    against the eager results."""
    w = WORKLOADS["ball3d_q3_64"]
    op = gpu_op(w)
    u = torch.from_numpy(uniform_vector(w.n_lattice, SEED_U)).cuda()
    wv = torch.from_numpy(uniform_vector(w.n_lattice, 21)).cuda()
    ref_du, ref_dg = op.vjp(u, wv)
    ref_c = op.cell_apply(u)
    du = torch.zeros_like(u)
    yc = torch.zeros_like(u)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        op.vjp(u, wv, du=du)
        op.cell_apply(u, yc)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _, dg = op.vjp(u, wv, du=du, accumulate=False)
        op.cell_apply(u, yc)
    for _ in range(3):
        du.fill_(5.0)
        yc.zero_()
        dg.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        sup = ref_du != 0
        assert float((du[sup] - ref_du[sup]).abs().max()) <= 1e-13 * float(ref_du.abs().max())
        assert float((dg - ref_dg).abs().max()) <= 1e-13 * float(ref_dg.abs().max())
        assert float((yc - ref_c).abs().max()) <= 1e-14 * float(ref_c.abs().max())


def test_destroy_returns_device_memory():
    """ghost_destroy frees every device allocation of a context (plan, tables, box layout, VJP and CG
    workspaces): free device memory is back where it started after repeated set-up, use and destroy."""
    from paper_2503_00246_amd.operator import GhostOperator
    w = WORKLOADS["ball3d_q3_64"]
    u = torch.from_numpy(uniform_vector(w.n_lattice, SEED_U)).cuda()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for i in range(6):
        op = GhostOperator.from_workload(w)
        y = op.apply(u)
        op.vjp(u, y)
        if i % 2 == 0:
            op.cg(torch.where(op.mass_diag() > 0, u, torch.zeros_like(u)), max_iter=3)
        torch.cuda.synchronize()
        op.close()
        del op, y
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 >= free0 - 64 * 2 ** 20, (free0, free1)
