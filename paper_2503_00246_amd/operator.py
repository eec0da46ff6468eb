"""Python face of libghost: GhostOperator and cg_solve.

PyTorch supplies device memory and the current HIP stream; every operation is
a call into the HIP library (include/ghost.h).
"""

import ctypes

import numpy as np

from . import _lib as L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class GhostOperator:
    """Matrix-free ghost penalty y = G(gamma) u on a Cartesian mesh cut by a level set.

    d, n, lo, h: mesh (cells per axis, lower corner, cell side); k: degree;
    gamma: k coefficients (penalty="derivative", the ghost penalty of derivative jumps) or one,
    gamma_M (penalty="macro", the macro-patch stabilisation); either (centre, radius) of a ball, balls (a sequence of
    (c0, c1, c2, r), their union), or cell_class (x-fastest array of 0 outside /
    1 inside / 2 cut).  device=-1 builds a
    host-only plan (inspection without a GPU).
    """

    SCATTERS = ("box", "atomic", "coloured")
    PENALTIES = ("derivative", "macro")

    def __init__(self, d, n, lo, h, k, gamma, centre=None, radius=None, cell_class=None,
                 scatter="box", device=0, balls=None, penalty="derivative"):
        lib = L.load()
        mesh = L.GhostMesh()
        mesh.dim = d
        for a in range(3):
            mesh.n[a] = int(n[a]) if a < d else 1
            mesh.lo[a] = float(lo[a]) if a < d else 0.0
        mesh.h = float(h)
        ls = L.GhostLevelset()
        self._cls_keep = None
        if cell_class is not None:
            ls.kind = L.GHOST_LS_CELLS
            arr = np.ascontiguousarray(np.asarray(cell_class, dtype=np.int8).ravel())
            self._cls_keep = arr
            ls.cell_class = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_byte))
        elif balls is not None:
            ls.kind = L.GHOST_LS_BALLS
            arr = np.ascontiguousarray(np.asarray(balls, dtype=np.float64).reshape(-1, 4))
            self._cls_keep = arr
            ls.n_balls = len(arr)
            ls.balls = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            ls.kind = L.GHOST_LS_BALL
            for a in range(3):
                ls.centre[a] = float(centre[a]) if a < d else 0.0
            ls.radius = float(radius)
        if penalty not in self.PENALTIES:
            raise ValueError(f"penalty must be one of {self.PENALTIES}")
        n_gamma = k if penalty == "derivative" else 1
        gamma = [float(x) for x in gamma]
        if len(gamma) != n_gamma:
            raise ValueError(f"need {n_gamma} coefficients for the {penalty} penalty")
        g = (ctypes.c_double * n_gamma)(*gamma)
        if scatter not in self.SCATTERS:
            raise ValueError(f"scatter must be one of {self.SCATTERS}")
        flags = L.GHOST_FP64 | L.GHOST_FP32 | {"box": 0, "atomic": L.GHOST_ATOMIC,
                                               "coloured": L.GHOST_COLOURED}[scatter]
        if penalty == "macro":
            flags |= L.GHOST_MACRO_PATCH
        self.scatter = scatter
        handle = ctypes.c_void_p()
        L.check(lib.ghost_setup(ctypes.byref(mesh), ctypes.byref(ls), int(k), g, flags, int(device),
                                ctypes.byref(handle)))
        self._h = handle
        self._lib = lib
        self.d, self.k, self.device = d, k, device
        self.penalty, self.n_gamma = penalty, n_gamma
        self.gamma = gamma
        st = L.GhostStats()
        L.check(lib.ghost_info(self._h, ctypes.byref(st)))
        self.stats = st.as_dict()
        self.n_lattice = self.stats["n_lattice"]

    @classmethod
    def from_workload(cls, w, scatter="box", device=0, gamma=None, penalty="derivative"):
        if gamma is None:
            gamma = w.gamma() if penalty == "derivative" else [w.gamma_macro()]
        return cls(w.d, w.n, w.lo, w.h, w.k, gamma, centre=w.centre, radius=w.radius, scatter=scatter,
                   device=device, balls=w.balls if w.balls else None, penalty=penalty)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ghost_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ checks
    def _vec(self, t, dtype, name):
        import torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if t.device.type != "cuda" or t.device.index != self.device:
            raise ValueError(f"{name} must live on cuda:{self.device}")
        if not t.is_contiguous() or t.numel() != self.n_lattice:
            raise ValueError(f"{name} must be contiguous with {self.n_lattice} entries")
        return t

    def _dev(self):
        import torch
        return torch.device("cuda", self.device)

    # ------------------------------------------------------------------ operations
    def apply(self, u, y=None, accumulate=False):
        """y (+)= G u in FP64.  Without y a zeroed output is allocated."""
        import torch
        self._vec(u, torch.float64, "u")
        if y is None:
            y = torch.zeros_like(u)
        self._vec(y, torch.float64, "y")
        L.check(self._lib.ghost_apply(self._h, _ptr(u), _ptr(y), int(accumulate), _stream(self._dev())))
        return y

    def cell_apply(self, u, y=None):
        """y += K_inside u: the Laplacian on the cells the boundary does not cut (float64 or float32,
        y allocated zeroed when omitted)."""
        import torch
        dt = u.dtype if isinstance(u, torch.Tensor) else None
        if dt not in (torch.float64, torch.float32):
            raise TypeError("u must be a float64 or float32 torch tensor")
        self._vec(u, dt, "u")
        if y is None:
            y = torch.zeros_like(u)
        self._vec(y, dt, "y")
        fn = self._lib.ghost_cell_apply if dt == torch.float64 else self._lib.ghost_cell_apply_f32
        L.check(fn(self._h, _ptr(u), _ptr(y), _stream(self._dev())))
        return y

    def face_bench(self, inp, out=None, reps=1):
        """Single-face microbenchmark: out = reps * G_F inp for every face of inp, a float64 or float32
        CUDA tensor of shape (n_faces, 2k+1, (k+1)^(d-1)) in the face's local layout [normal node][line]."""
        import torch
        n_p = (2 * self.k + 1) * (self.k + 1) ** (self.d - 1)
        if not isinstance(inp, torch.Tensor) or inp.dtype not in (torch.float64, torch.float32):
            raise TypeError("inp must be a float64 or float32 torch tensor")
        if inp.device.type != "cuda" or inp.device.index != self.device or not inp.is_contiguous():
            raise ValueError(f"inp must be contiguous on cuda:{self.device}")
        if inp.numel() % n_p:
            raise ValueError(f"inp must hold whole faces of {n_p} values")
        if out is None:
            out = torch.empty_like(inp)
        if out.dtype != inp.dtype or out.shape != inp.shape or not out.is_contiguous():
            raise ValueError("out must match inp")
        fn = self._lib.ghost_face_bench if inp.dtype == torch.float64 else self._lib.ghost_face_bench_f32
        L.check(fn(self._h, _ptr(inp), _ptr(out), inp.numel() // n_p, int(reps), _stream(self._dev())))
        return out

    def apply_f32(self, u, y=None, accumulate=False):
        import torch
        self._vec(u, torch.float32, "u")
        if y is None:
            y = torch.zeros_like(u)
        self._vec(y, torch.float32, "y")
        L.check(self._lib.ghost_apply_f32(self._h, _ptr(u), _ptr(y), int(accumulate), _stream(self._dev())))
        return y

    def vjp(self, u, w, du=None, accumulate=False):
        """(G w, [w^T G_j u]_j) for the pull-back of w through y = G(gamma) u."""
        import torch
        self._vec(u, torch.float64, "u")
        self._vec(w, torch.float64, "w")
        if du is None:
            du = torch.zeros_like(u)
        self._vec(du, torch.float64, "du")
        dg = torch.empty(self.n_gamma, dtype=torch.float64, device=self._dev())
        L.check(self._lib.ghost_vjp(self._h, _ptr(u), _ptr(w), _ptr(du), _ptr(dg), int(accumulate),
                                    _stream(self._dev())))
        return du, dg

    def set_gamma(self, gamma):
        """Replace gamma: a host sequence (validated) or a float64 CUDA tensor of n_gamma values
        (stream-ordered)."""
        import torch
        if isinstance(gamma, torch.Tensor) and gamma.device.type == "cuda":
            if gamma.dtype != torch.float64 or gamma.numel() != self.n_gamma or not gamma.is_contiguous():
                raise ValueError(f"device gamma must be a contiguous float64 tensor of {self.n_gamma} values")
            L.check(self._lib.ghost_set_gamma(self._h, _ptr(gamma), 1, _stream(self._dev())))
            return
        vals = [float(x) for x in (gamma.tolist() if hasattr(gamma, "tolist") else gamma)]
        if len(vals) != self.n_gamma:
            raise ValueError(f"need {self.n_gamma} coefficients")
        arr = (ctypes.c_double * self.n_gamma)(*vals)
        L.check(self._lib.ghost_set_gamma(self._h, ctypes.cast(arr, ctypes.c_void_p), 0, _stream(self._dev())))
        self.gamma = vals

    def ghost_diag(self, out=None, accumulate=False):
        """Diagonal of G (FP64, on the support; other entries of a fresh output are 0)."""
        import torch
        if out is None:
            out = torch.zeros(self.n_lattice, dtype=torch.float64, device=self._dev())
        self._vec(out, torch.float64, "diag")
        L.check(self._lib.ghost_diag(self._h, _ptr(out), int(accumulate), _stream(self._dev())))
        return out

    def mass_diag(self):
        import torch
        out = torch.empty(self.n_lattice, dtype=torch.float64, device=self._dev())
        L.check(self._lib.ghost_mass_diag(self._h, _ptr(out), _stream(self._dev())))
        return out

    def cg(self, b, x=None, mode="fp64", tol=1e-10, max_iter=20000, inner_tol=1e-4, check_every=50, precond="none"):
        """Solve (M + G) x = b on the active nodes; returns (x, result dict).  Synchronous.
        precond: "none" or "jacobi" (diagonal of M + G)."""
        import torch
        self._vec(b, torch.float64, "b")
        if x is None:
            x = torch.zeros_like(b)
        self._vec(x, torch.float64, "x")
        opts = L.GhostCgOpts()
        opts.mode = {"fp64": L.GHOST_CG_FP64, "mixed": L.GHOST_CG_MIXED}[mode]
        opts.tol, opts.max_iter, opts.inner_tol, opts.check_every = tol, max_iter, inner_tol, check_every
        opts.precond = {"none": L.GHOST_CG_NONE, "jacobi": L.GHOST_CG_JACOBI}[precond]
        res = L.GhostCgResult()
        L.check(self._lib.ghost_cg(self._h, _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(res),
                                   _stream(self._dev())))
        return x, {"iterations": res.iterations, "outer": res.outer, "converged": bool(res.converged),
                   "rel_residual": res.rel_residual}

    # ------------------------------------------------------------------ inspection (host)
    def faces(self, axis):
        """(nf, 4) int32: lower-cell multi-index c0, c1, c2 and colour (-1 if not coloured)."""
        nf = self.stats["n_faces"][axis]
        out = np.zeros((max(nf, 1), 4), dtype=np.int32)
        L.check(self._lib.ghost_faces(self._h, axis, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nf))
        return out[:nf]

    def box_layout(self):
        """Box-scatter layout: (boxes (nb, 7) int32, visits uint64, runs (nr, 4) int64)."""
        nb, nv = self.stats["n_boxes"], self.stats["n_visits"]
        boxes = np.zeros((max(nb, 1), 7), dtype=np.int32)
        visits = np.zeros(max(nv, 1), dtype=np.uint64)
        L.check(self._lib.ghost_box_layout(self._h, boxes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nb,
                                           visits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), nv, None, 0))
        boxes = boxes[:nb]
        nr = int((boxes[:, 5] + boxes[:, 6]).max()) if nb else 0
        runs = np.zeros((max(nr, 1), 4), dtype=np.int64)
        L.check(self._lib.ghost_box_layout(self._h, None, 0, None, 0,
                                           runs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nr))
        return boxes, visits[:nv], runs[:nr]

    def cell_chunks(self):
        """Chunks of the interior Laplacian: (n, 3) int64 of (first node, cell count, colour)."""
        n = self.stats["n_cell_chunks"]
        out = np.zeros((max(n, 1), 3), dtype=np.int64)
        L.check(self._lib.ghost_cell_chunks(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n))
        return out[:n]

    def set_timing(self, on=True):
        """Record per-kernel HIP events in later applies / VJPs (see kernel_times)."""
        L.check(self._lib.ghost_set_timing(self._h, 1 if on else 0))

    def kernel_times(self):
        """Summed durations (ms) of the scatter kernels and of the halo pass over the calls recorded
        since the last read, and the number of calls; waits for the recorded events."""
        a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        L.check(self._lib.ghost_kernel_times(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)))
        return {"main_ms": a.value, "halo_ms": b.value, "calls": n.value}

    def tables(self):
        k = self.k
        jumps = np.zeros((k, 2 * k + 1))
        mass = np.zeros((k + 1, k + 1))
        nodes = np.zeros(k + 1)
        weights = np.zeros(k + 1)
        dp = ctypes.POINTER(ctypes.c_double)
        L.check(self._lib.ghost_tables(self._h, jumps.ctypes.data_as(dp), mass.ctypes.data_as(dp),
                                       nodes.ctypes.data_as(dp), weights.ctypes.data_as(dp)))
        return {"jumps": jumps, "mass": mass, "nodes": nodes, "weights": weights}


def cg_solve(op, b, mode="fp64", **kw):
    return op.cg(b, mode=mode, **kw)
