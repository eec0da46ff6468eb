"""ctypes binding of libghost (include/ghost.h): structures, prototypes and error checking.

Argument marshalling only; every operation runs in the HIP library.  Loading
fails loudly when the library has not been built -- there is no fallback.
"""

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libghost.so")

GHOST_OK, GHOST_EINVAL, GHOST_ENOMEM, GHOST_EHIP, GHOST_ESTATE = 0, -1, -2, -3, -4
GHOST_KMAX = 7
GHOST_LS_BALL, GHOST_LS_CELLS, GHOST_LS_BALLS = 0, 1, 2
GHOST_FP64, GHOST_FP32, GHOST_COLOURED, GHOST_ATOMIC, GHOST_MACRO_PATCH = 1, 2, 4, 8, 16
GHOST_CG_FP64, GHOST_CG_MIXED = 0, 1
GHOST_CG_NONE, GHOST_CG_JACOBI = 0, 1

EXPORTS = ["ghost_setup", "ghost_set_gamma", "ghost_apply", "ghost_apply_f32", "ghost_vjp",
           "ghost_mass_diag", "ghost_cg", "ghost_info", "ghost_faces", "ghost_tables", "ghost_box_layout",
           "ghost_destroy", "ghost_last_error", "ghost_set_timing", "ghost_kernel_times", "ghost_diag",
           "ghost_face_bench", "ghost_face_bench_f32", "ghost_cell_apply", "ghost_cell_apply_f32",
           "ghost_cell_chunks"]


class GhostMesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("h", ctypes.c_double)]


class GhostLevelset(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("centre", ctypes.c_double * 3), ("radius", ctypes.c_double),
                ("cell_class", ctypes.POINTER(ctypes.c_byte)), ("n_balls", ctypes.c_int),
                ("balls", ctypes.POINTER(ctypes.c_double))]


class GhostStats(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("k", ctypes.c_int), ("device", ctypes.c_int), ("n_colours", ctypes.c_int),
                ("lattice", ctypes.c_int64 * 3), ("n_lattice", ctypes.c_int64),
                ("n_cells", ctypes.c_int64), ("n_active_cells", ctypes.c_int64), ("n_cut_cells", ctypes.c_int64),
                ("n_active_dofs", ctypes.c_int64), ("n_support_dofs", ctypes.c_int64),
                ("n_faces", ctypes.c_int64 * 3), ("n_faces_total", ctypes.c_int64),
                ("n_patch_dofs", ctypes.c_int64), ("n_batches", ctypes.c_int64),
                ("n_boxes", ctypes.c_int64), ("n_visits", ctypes.c_int64), ("n_halo_slots", ctypes.c_int64),
                ("n_halo_nodes", ctypes.c_int64), ("brick", ctypes.c_int),
                ("flops_per_face", ctypes.c_double), ("bytes_fp64", ctypes.c_double),
                ("bytes_fp32", ctypes.c_double), ("n_inside_dofs", ctypes.c_int64),
                ("n_gamma", ctypes.c_int), ("macro", ctypes.c_int), ("n_cell_chunks", ctypes.c_int64)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, ctypes.Array) else v
        return out


class GhostCgOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("check_every", ctypes.c_int), ("precond", ctypes.c_int)]


class GhostCgResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double)]


class GhostError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libghost error {code}: {msg}")
        self.code = code


_lib = None


def load(path=LIB_PATH):
    """Load the library once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not built: run `python -m paper_2503_00246_amd._build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, c_int, c_i64, c_u = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint
    lib.ghost_setup.argtypes = [ctypes.POINTER(GhostMesh), ctypes.POINTER(GhostLevelset), c_int,
                                ctypes.POINTER(ctypes.c_double), c_u, c_int, ctypes.POINTER(P)]
    lib.ghost_set_gamma.argtypes = [P, P, c_int, P]
    lib.ghost_apply.argtypes = [P, P, P, c_int, P]
    lib.ghost_apply_f32.argtypes = [P, P, P, c_int, P]
    lib.ghost_vjp.argtypes = [P, P, P, P, P, c_int, P]
    lib.ghost_mass_diag.argtypes = [P, P, P]
    lib.ghost_diag.argtypes = [P, P, c_int, P]
    lib.ghost_face_bench.argtypes = [P, P, P, c_i64, c_int, P]
    lib.ghost_cell_apply.argtypes = [P, P, P, P]
    lib.ghost_cell_apply_f32.argtypes = [P, P, P, P]
    lib.ghost_cell_chunks.argtypes = [P, ctypes.POINTER(ctypes.c_int64), c_i64]
    lib.ghost_face_bench_f32.argtypes = [P, P, P, c_i64, c_int, P]
    lib.ghost_cg.argtypes = [P, P, P, ctypes.POINTER(GhostCgOpts), ctypes.POINTER(GhostCgResult), P]
    lib.ghost_info.argtypes = [P, ctypes.POINTER(GhostStats)]
    lib.ghost_faces.argtypes = [P, c_int, ctypes.POINTER(ctypes.c_int32), c_i64]
    lib.ghost_tables.argtypes = [P] + [ctypes.POINTER(ctypes.c_double)] * 4
    lib.ghost_box_layout.argtypes = [P, ctypes.POINTER(ctypes.c_int32), c_i64, ctypes.POINTER(ctypes.c_uint64),
                                     c_i64, ctypes.POINTER(ctypes.c_int64), c_i64]
    lib.ghost_set_timing.argtypes = [P, c_int]
    lib.ghost_kernel_times.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(c_i64)]
    lib.ghost_destroy.argtypes = [P]
    lib.ghost_destroy.restype = None
    lib.ghost_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("ghost_destroy", "ghost_last_error"):
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def check(rc):
    if rc != GHOST_OK:
        msg = _lib.ghost_last_error().decode(errors="replace") if _lib is not None else ""
        raise GhostError(rc, msg)
    return rc
