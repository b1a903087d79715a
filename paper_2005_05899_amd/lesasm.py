"""Thin ctypes binding of the C-ABI library ``_lib/liblesasm.so``.

Argument marshalling only: every step of the assembly runs in the library's
HIP kernels.  PyTorch provides device memory (tensors) and the current HIP
stream.  If the library is missing this module raises on use; there is no
fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (load torch's HIP runtime before the library binds to it)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "liblesasm.so")

OK, E_INVALID_ARG, E_INVERTED_ELEMENT, E_OOM, E_HIP, E_STATE, E_NONFINITE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
TET04, PYR05, PEN06, HEX08 = 4, 5, 6, 8
MESH_SCATTER_STAGED, MESH_SCATTER_COLOUR, MESH_KEEP_ORDER, MESH_SCATTER_DIRECT, MESH_SCATTER_CHUNK_ATOMIC = 0, 1, 2, 4, 8
OPT_PRECISION, OPT_RHS_MODE, OPT_CHECK_FINITE, OPT_BLOCK, OPT_PROFILE, OPT_CHUNK, OPT_CONCURRENT = 1, 2, 3, 4, 5, 6, 7
OPT_PERSISTENT = 8
KERNEL_SLOTS = ("fill", "tet04", "pyr05", "pen06", "hex08", "increment", "gather")
PREC_FP64, PREC_FP32 = 0, 1
RHS_RESIDUAL, RHS_INCREMENT = 0, 1

# every symbol declared in include/lesasm.h
EXPORTS = [
    "lesasm_mesh_create", "lesasm_mesh_destroy", "lesasm_mesh_get_info", "lesasm_mesh_node_permutation",
    "lesasm_mesh_element_permutation", "lesasm_fields_to_internal", "lesasm_fields_to_user",
    "lesasm_mesh_lumped_mass", "lesasm_mesh_filter_width", "lesasm_mesh_set_option", "lesasm_mesh_get_option",
    "lesasm_assemble_momentum_rhs", "lesasm_mesh_kernel_times", "lesasm_last_error", "lesasm_version",
    "lesasm_check", "lesasm_mesh_set_wall", "lesasm_assemble_wall",
    "lesasm_divergence", "lesasm_gradient", "lesasm_stepper_create", "lesasm_stepper_destroy", "lesasm_stepper_step",
    "lesasm_stepper_rk3_stages", "lesasm_pressure_solve", "lesasm_stepper_stats", "lesasm_stepper_laplacian",
    "lesasm_stepper_spmv", "lesasm_stepper_sell_entries",
    "lesasm_batch_create", "lesasm_batch_destroy", "lesasm_batch_configure", "lesasm_batch_get_config",
    "lesasm_batch_assemble", "lesasm_batch_tune", "lesasm_batch_rk3_graph", "lesasm_batch_rk3_launch",
    "lesasm_batch_rk3_eager", "lesasm_mlp_create", "lesasm_mlp_destroy", "lesasm_mlp_get_params",
    "lesasm_mlp_set_params", "lesasm_mlp_loss_grad", "lesasm_mlp_adam", "lesasm_mlp_train_step", "lesasm_mlp_commit",
    "lesasm_mlp_forward_f32", "lesasm_mlp_infer_bf16", "lesasm_mesh_set_closure", "lesasm_mesh_closure_fallbacks",
    "lesasm_mesh_closure_fallbacks_by_type",
    "lesasm_element_centroids", "lesasm_sfc_workspace_bytes", "lesasm_sfc_partition", "lesasm_balance_update",
    "lesasm_batch_set_per_type", "lesasm_batch_get_per_type",
    "lesasm_step_graph_create", "lesasm_step_graph_launch", "lesasm_step_graph_stats", "lesasm_step_graph_destroy",
    "lesasm_set_memory_cap", "lesasm_memory_in_use", "lesasm_mlp_loss_grad_noalloc",
]
MLP_PARAMS = 5254
ORDER_MESH, ORDER_LARGEST_FIRST, ORDER_INTERLEAVED = 0, 1, 2


# Library objects dropped by the garbage collector are not destroyed from the
# collector: a destroy synchronises the device, which must not happen while the
# caller is capturing a stream.  __del__ only queues the handle; queued handles
# are destroyed at the next object creation or explicit close() and at exit,
# step graphs before steppers before batches before meshes before networks.
_DESTROY_ORDER = {"lesasm_step_graph_destroy": 0, "lesasm_stepper_destroy": 1, "lesasm_batch_destroy": 2,
                  "lesasm_mesh_destroy": 3, "lesasm_mlp_destroy": 4}
_deferred: list = []


def _defer(fn: str, h) -> None:
    _deferred.append((_DESTROY_ORDER[fn], len(_deferred), fn, h))


def release_deferred() -> None:
    """Destroy the library objects the garbage collector has dropped."""
    if not _deferred:
        return
    items = sorted(_deferred)
    _deferred.clear()
    lib = load()
    for _, _, fn, h in items:
        getattr(lib, fn)(h)


atexit.register(release_deferred)


class LesasmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lesasm error {code}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64), ("coords", ctypes.c_void_p), ("n_elems", ctypes.c_int64),
        ("types", ctypes.c_void_p), ("conn_offsets", ctypes.c_void_p), ("conn", ctypes.c_void_p),
        ("field_node", ctypes.c_void_p), ("n_field_nodes", ctypes.c_int64), ("vreman_c", ctypes.c_double),
        ("flags", ctypes.c_uint32),
    ]


class WallDesc(ctypes.Structure):
    _fields_ = [("n_faces", ctypes.c_int64), ("face_offsets", ctypes.c_void_p), ("face_conn", ctypes.c_void_p),
                ("face_elem", ctypes.c_void_p)]


class MeshInfo(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64), ("n_field_nodes", ctypes.c_int64), ("n_elems", ctypes.c_int64),
        ("n_per_type", ctypes.c_int64 * 4), ("n_colours", ctypes.c_int32 * 4), ("device", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2005_05899_amd/build.py")
    lib = ctypes.CDLL(path)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "lesasm_mesh_create": [P, P], "lesasm_mesh_destroy": [P], "lesasm_mesh_get_info": [P, P],
        "lesasm_mesh_node_permutation": [P, P], "lesasm_mesh_element_permutation": [P, P],
        "lesasm_fields_to_internal": [P, P, P, I, P], "lesasm_fields_to_user": [P, P, P, I, P],
        "lesasm_mesh_lumped_mass": [P, P, P], "lesasm_mesh_filter_width": [P, P, P],
        "lesasm_mesh_set_option": [P, I, I64], "lesasm_mesh_get_option": [P, I, P],
        "lesasm_assemble_momentum_rhs": [P, P, P, D, D, P, P], "lesasm_mesh_kernel_times": [P, P, P, I],
        "lesasm_version": [], "lesasm_check": [P], "lesasm_mesh_set_wall": [P, P],
        "lesasm_assemble_wall": [P, P, D, P, P], "lesasm_divergence": [P, P, P, P], "lesasm_gradient": [P, P, P, P],
        "lesasm_stepper_create": [P, D, D, D, I, P], "lesasm_stepper_destroy": [P], "lesasm_stepper_step": [P, P, P, P],
        "lesasm_stepper_rk3_stages": [P, P, P, P, P], "lesasm_pressure_solve": [P, P, P, P],
        "lesasm_stepper_stats": [P, P, P], "lesasm_stepper_laplacian": [P, P, P, P, P],
        "lesasm_stepper_spmv": [P, P, P, P], "lesasm_stepper_sell_entries": [P, P],
        "lesasm_batch_create": [P, I, P], "lesasm_batch_destroy": [P], "lesasm_batch_configure": [P, I, I, I],
        "lesasm_batch_get_config": [P, P, P, P, P], "lesasm_batch_assemble": [P, P, P, P, P, P],
        "lesasm_batch_tune": [P, P, P, P, P, ctypes.c_char_p, I, P], "lesasm_batch_rk3_graph": [P, P, P, P, D, P],
        "lesasm_batch_rk3_launch": [P, P], "lesasm_batch_rk3_eager": [P, P, P, P, D, P],
        "lesasm_mlp_create": [P, P], "lesasm_mlp_destroy": [P], "lesasm_mlp_get_params": [P, P],
        "lesasm_mlp_set_params": [P, P], "lesasm_mlp_loss_grad": [P, P, P, I, P, P, P],
        "lesasm_mlp_loss_grad_noalloc": [P, P, P, I, P, P, P],
        "lesasm_mlp_adam": [P, P, ctypes.c_float, P], "lesasm_mlp_train_step": [P, P, P, I, ctypes.c_float, P, P],
        "lesasm_mlp_commit": [P], "lesasm_mlp_forward_f32": [P, P, I, P, P], "lesasm_mlp_infer_bf16": [P, P, I, P, P],
        "lesasm_mesh_set_closure": [P, P, D, D], "lesasm_mesh_closure_fallbacks": [P, P],
        "lesasm_mesh_closure_fallbacks_by_type": [P, P],
        "lesasm_element_centroids": [I64, P, P, I64, I64, P, P, P, P, P],
        "lesasm_sfc_workspace_bytes": [I64, I, I, P], "lesasm_sfc_partition": [I64, P, P, I, P, I, P, ctypes.c_size_t, P, P],
        "lesasm_balance_update": [I, I, P, P, D, P],
        "lesasm_batch_set_per_type": [P, I], "lesasm_batch_get_per_type": [P, P],
        "lesasm_step_graph_create": [P, P, P, I, P, P], "lesasm_step_graph_launch": [P, P, P, P],
        "lesasm_step_graph_stats": [P, P, P, P], "lesasm_step_graph_destroy": [P],
        "lesasm_set_memory_cap": [ctypes.c_uint64], "lesasm_memory_in_use": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.lesasm_last_error.argtypes = []
    lib.lesasm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int):
    if status != OK:
        raise LesasmError(status, load().lesasm_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    """A mesh uploaded to the current GPU (see lesasm_mesh_create)."""

    def __init__(self, coords, types, conn_offsets, conn, field_node=None, n_field_nodes=0,
                 vreman_c: float = 0.1, colour: bool = False, keep_order: bool = False,
                 scatter: str | None = None):
        """scatter: "staged" (default), "chunk_atomic", "colour" or "direct"; colour=True is "colour"."""
        release_deferred()
        lib = load()
        self._keep = [np.ascontiguousarray(coords, np.float64), np.ascontiguousarray(types, np.uint8),
                      np.ascontiguousarray(conn_offsets, np.int64), np.ascontiguousarray(conn, np.int32),
                      None if field_node is None else np.ascontiguousarray(field_node, np.int32)]
        c, t, o, cn, fn = self._keep
        d = MeshDesc(len(c), c.ctypes.data, len(t), t.ctypes.data, o.ctypes.data, cn.ctypes.data,
                     None if fn is None else fn.ctypes.data, int(n_field_nodes) if fn is not None else 0,
                     float(vreman_c), self._flags(scatter or ("colour" if colour else "staged"), keep_order))
        h = ctypes.c_void_p()
        check(lib.lesasm_mesh_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._keep = None
        info = MeshInfo()
        check(lib.lesasm_mesh_get_info(self._h, ctypes.byref(info)))
        self.n_nodes, self.n_field_nodes, self.n_elems = info.n_nodes, info.n_field_nodes, info.n_elems
        self.n_per_type = dict(zip((TET04, PYR05, PEN06, HEX08), list(info.n_per_type)))
        self.n_colours = dict(zip((TET04, PYR05, PEN06, HEX08), list(info.n_colours)))
        self.device_index = info.device
        self.device_bytes = info.device_bytes
        self.device = torch.device("cuda", info.device)

    @staticmethod
    def _flags(scatter: str, keep_order: bool) -> int:
        f = {"staged": MESH_SCATTER_STAGED, "chunk_atomic": MESH_SCATTER_CHUNK_ATOMIC, "colour": MESH_SCATTER_COLOUR,
             "direct": MESH_SCATTER_DIRECT}[scatter]
        return f | (MESH_KEEP_ORDER if keep_order else 0)

    @classmethod
    def from_arrays(cls, m, vreman_c: float = 0.1, **kw) -> "Mesh":
        """From any object with coords / types / conn_offsets / conn / field_node / n_field_nodes."""
        return cls(m.coords, m.types, m.conn_offsets, m.conn, m.field_node, m.n_field_nodes, vreman_c, **kw)

    def close(self):
        if getattr(self, "_h", None):
            load().lesasm_mesh_destroy(self._h)
            self._h = None
        release_deferred()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _defer("lesasm_mesh_destroy", h)

    # ---- orderings ---------------------------------------------------------
    def node_permutation(self) -> np.ndarray:
        perm = np.empty(self.n_field_nodes, np.int32)
        check(load().lesasm_mesh_node_permutation(self._h, perm.ctypes.data))
        return perm

    def element_permutation(self) -> np.ndarray:
        perm = np.empty(self.n_elems, np.int64)
        check(load().lesasm_mesh_element_permutation(self._h, perm.ctypes.data))
        return perm

    def _field(self, t, ncomp=None):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("expected a contiguous float64 tensor on the GPU")
        if t.shape[0] != self.n_field_nodes:
            raise ValueError(f"expected {self.n_field_nodes} rows, got {t.shape[0]}")
        return t if ncomp is None else t

    def to_internal(self, t):
        t = self._field(t)
        out = torch.empty_like(t)
        nc = 1 if t.dim() == 1 else int(np.prod(t.shape[1:]))
        check(load().lesasm_fields_to_internal(self._h, _ptr(t), _ptr(out), nc, _stream()))
        return out

    def to_user(self, t):
        t = self._field(t)
        out = torch.empty_like(t)
        nc = 1 if t.dim() == 1 else int(np.prod(t.shape[1:]))
        check(load().lesasm_fields_to_user(self._h, _ptr(t), _ptr(out), nc, _stream()))
        return out

    def lumped_mass(self):
        out = torch.empty(self.n_field_nodes, dtype=torch.float64, device=self.device)
        check(load().lesasm_mesh_lumped_mass(self._h, _ptr(out), _stream()))
        return out

    def filter_width(self):
        out = torch.empty(self.n_elems, dtype=torch.float64, device=self.device)
        check(load().lesasm_mesh_filter_width(self._h, _ptr(out), _stream()))
        return out

    # ---- options -----------------------------------------------------------
    def set_option(self, option: int, value: int):
        check(load().lesasm_mesh_set_option(self._h, option, int(value)))

    def get_option(self, option: int) -> int:
        v = ctypes.c_int64()
        check(load().lesasm_mesh_get_option(self._h, option, ctypes.byref(v)))
        return v.value

    @property
    def precision(self) -> str:
        return "fp32" if self.get_option(OPT_PRECISION) == PREC_FP32 else "fp64"

    @precision.setter
    def precision(self, value: str):
        self.set_option(OPT_PRECISION, {"fp64": PREC_FP64, "fp32": PREC_FP32}[value])

    def kernel_times(self, reset: bool = False) -> dict:
        """{slot: (total ms, launches)} from the events recorded with OPT_PROFILE."""
        ms = (ctypes.c_double * len(KERNEL_SLOTS))()
        n = (ctypes.c_int64 * len(KERNEL_SLOTS))()
        check(load().lesasm_mesh_kernel_times(self._h, ms, n, int(reset)))
        return {k: (ms[i], n[i]) for i, k in enumerate(KERNEL_SLOTS)}

    # ---- the hot path --------------------------------------------------------
    def set_wall(self, face_offsets, face_conn, face_elem):
        """Wall faces (user node and element ids) for the wall model."""
        fo = np.ascontiguousarray(face_offsets, dtype=np.int64)
        fc = np.ascontiguousarray(face_conn, dtype=np.int32)
        fe = np.ascontiguousarray(face_elem, dtype=np.int64)
        d = WallDesc(len(fe), fo.ctypes.data, fc.ctypes.data, fe.ctypes.data)
        check(load().lesasm_mesh_set_wall(self._h, ctypes.byref(d)))

    def assemble_wall(self, u, nu: float, out):
        """out += wall-model contributions (internal order)."""
        u = self._field(u)
        check(load().lesasm_assemble_wall(self._h, _ptr(u), float(nu), _ptr(out), _stream()))
        return out

    def assemble_momentum_rhs(self, u, p=None, nu: float = 0.0, dt: float = 0.0, out=None):
        """rhs [n_field_nodes, 3] (internal order) of M_L du/dt = rhs for velocity
        u [n_field_nodes, 3] and modified pressure p [n_field_nodes] (or None)."""
        u = self._field(u)
        if p is not None:
            p = self._field(p)
        if out is None:
            out = torch.empty((self.n_field_nodes, 3), dtype=torch.float64, device=u.device)
        check(load().lesasm_assemble_momentum_rhs(self._h, _ptr(u), _ptr(p), float(nu), float(dt), _ptr(out),
                                                  _stream()))
        return out


class Stepper:
    """Fractional-step time integration on a mesh (lesasm_stepper_*)."""

    def __init__(self, mesh: Mesh, nu: float, dt: float, rtol: float = 1e-12, maxit: int = 2000):
        release_deferred()
        self.mesh = mesh
        h = ctypes.c_void_p()
        check(load().lesasm_stepper_create(mesh._h, float(nu), float(dt), float(rtol), int(maxit), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().lesasm_stepper_destroy(self._h)
            self._h = None
        release_deferred()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _defer("lesasm_stepper_destroy", h)

    def step(self, u, p):
        """One time step in place on internal-order tensors u [n,3], p [n]."""
        self.mesh._field(u)
        self.mesh._field(p)
        check(load().lesasm_stepper_step(self._h, _ptr(u), _ptr(p), _stream()))

    def rk3_stages(self, u, p):
        out = torch.empty_like(u)
        check(load().lesasm_stepper_rk3_stages(self._h, _ptr(u), _ptr(p), _ptr(out), _stream()))
        return out

    def pressure_solve(self, b):
        x = torch.empty_like(b)
        check(load().lesasm_pressure_solve(self._h, _ptr(b), _ptr(x), _stream()))
        return x

    def stats(self):
        it, res = ctypes.c_int(), ctypes.c_double()
        check(load().lesasm_stepper_stats(self._h, ctypes.byref(it), ctypes.byref(res)))
        return it.value, res.value

    def spmv(self, p, out=None):
        """q = K p (internal order) by the pressure CG's product kernel."""
        self.mesh._field(p)
        if p.numel() != self.mesh.n_field_nodes:
            raise ValueError("expected one value per field node")
        q = torch.empty_like(p) if out is None else self.mesh._field(out)
        if q.numel() != p.numel():
            raise ValueError("out must match p")
        check(load().lesasm_stepper_spmv(self._h, _ptr(p), _ptr(q), _stream()))
        return q

    def sell_entries(self) -> int:
        """Stored entries (nonzeros plus padding) of the sliced-ELLPACK copy of K."""
        e = ctypes.c_int64()
        check(load().lesasm_stepper_sell_entries(self._h, ctypes.byref(e)))
        return e.value

    def laplacian(self):
        """(rowptr, col, val) host arrays of the assembled K (internal order)."""
        nnz = ctypes.c_int64()
        check(load().lesasm_stepper_laplacian(self._h, None, None, None, ctypes.byref(nnz)))
        rowptr = np.empty(self.mesh.n_field_nodes + 1, np.int32)
        col = np.empty(nnz.value, np.int32)
        val = np.empty(nnz.value, np.float64)
        check(load().lesasm_stepper_laplacian(self._h, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data,
                                              ctypes.byref(nnz)))
        return rowptr, col, val


def set_memory_cap(nbytes: int):
    """Cap on the device memory the library allocates (0: none)."""
    check(load().lesasm_set_memory_cap(int(nbytes)))


def memory_in_use() -> int:
    """Device bytes the library holds now."""
    v = ctypes.c_uint64()
    check(load().lesasm_memory_in_use(ctypes.byref(v)))
    return v.value


class StepGraph:
    """One whole time step of a Stepper captured in a HIP graph
    (lesasm_step_graph_*), bound to the tensors u [n,3] and p [n] (internal
    order), which every replay updates in place."""

    def __init__(self, stepper: "Stepper", u, p, cg_iters: int, stream):
        release_deferred()
        stepper.mesh._field(u)
        stepper.mesh._field(p)
        self.stepper, self.u, self.p = stepper, u, p
        h = ctypes.c_void_p()
        check(load().lesasm_step_graph_create(stepper._h, _ptr(u), _ptr(p), int(cg_iters), ctypes.byref(h),
                                              stream.cuda_stream))
        self._h = h

    def launch(self, stream=None, u=None, p=None):
        """Replay on `stream` (default: torch's current stream).  Passing other
        tensors than the bound ones is rejected by the library."""
        u = self.u if u is None else u
        p = self.p if p is None else p
        s = _stream() if stream is None else stream.cuda_stream
        check(load().lesasm_step_graph_launch(self._h, _ptr(u), _ptr(p), s))

    def stats(self):
        """(CG iterations, relative residual, converged) of the last replay."""
        it, res, ok = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
        check(load().lesasm_step_graph_stats(self._h, ctypes.byref(it), ctypes.byref(res), ctypes.byref(ok)))
        return it.value, res.value, bool(ok.value)

    def close(self):
        if getattr(self, "_h", None):
            check(load().lesasm_step_graph_destroy(self._h))
            self._h = None
        release_deferred()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _defer("lesasm_step_graph_destroy", h)


def check_stream(stream=None):
    """Wait for the stream (default: the current torch stream) and raise if an
    asynchronous library call failed on it."""
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    check(load().lesasm_check(s))


def divergence(mesh: Mesh, u):
    out = torch.empty(mesh.n_field_nodes, dtype=torch.float64, device=u.device)
    check(load().lesasm_divergence(mesh._h, _ptr(u), _ptr(out), _stream()))
    return out


def gradient(mesh: Mesh, p):
    out = torch.empty((mesh.n_field_nodes, 3), dtype=torch.float64, device=p.device)
    check(load().lesasm_gradient(mesh._h, _ptr(p), _ptr(out), _stream()))
    return out


# ---- SFC partitioning and load balancing ----------------------------------

def element_centroids(conn_offsets, conn, coords, weights=True, check_input=True, out=None):
    """(centroids [n,3] f64, Gauss-point weights [n] int32 or None) of the
    elements given by device tensors conn_offsets (int64), conn (int32) and
    coords ([n_nodes,3] f64), computed by lesasm_element_centroids.  With
    check_input the call waits for the stream and raises on invalid input.
    out = (centroids, weights or None, status int32 [1], zeroed by the caller)
    reuses buffers."""
    for t, dt in ((conn_offsets, torch.int64), (conn, torch.int32), (coords, torch.float64)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError("element_centroids: expects contiguous device tensors (int64, int32, float64)")
    n = max(conn_offsets.numel() - 1, 0)
    if out is not None:
        cen, w, status = out
        if cen.shape != (n, 3) or cen.dtype != torch.float64 or (w is not None and w.shape != (n,)) \
                or status.dtype != torch.int32:
            raise ValueError("element_centroids: output buffers of the wrong shape or type")
    else:
        cen = torch.empty((n, 3), dtype=torch.float64, device=coords.device)
        w = torch.empty(n, dtype=torch.int32, device=coords.device) if weights else None
        status = torch.zeros(1, dtype=torch.int32, device=coords.device)
    check(load().lesasm_element_centroids(n, _ptr(conn_offsets), _ptr(conn), conn.numel(), coords.shape[0],
                                          _ptr(coords), _ptr(cen), None if w is None else _ptr(w), _ptr(status),
                                          _stream()))
    if check_input:
        bad = int(status.item())
        if bad:
            raise LesasmError(-1, "element_centroids: " + ("an element has not 4, 5, 6 or 8 nodes or lies outside "
                                                           "conn" if bad & 1 else "node id out of range"))
    return cen, w


def sfc_partition(centroids, weights, n_parts: int, lam=None, level: int = 7, work=None):
    """Part (int32 device tensor) of every element: lesasm_sfc_partition on
    device tensors centroids [n,3] f64 and weights [n] int32 (or None);
    lam is a host sequence of n_parts correction coefficients or None."""
    if not centroids.is_cuda or centroids.dtype != torch.float64 or not centroids.is_contiguous():
        raise ValueError("sfc_partition: centroids must be a contiguous float64 device tensor")
    if weights is not None and (not weights.is_cuda or weights.dtype != torch.int32 or not weights.is_contiguous()
                                or weights.numel() != centroids.shape[0]):
        raise ValueError("sfc_partition: weights must be a contiguous int32 device tensor, one per element")
    n = centroids.shape[0]
    nbytes = ctypes.c_size_t()
    check(load().lesasm_sfc_workspace_bytes(n, int(n_parts), int(level), ctypes.byref(nbytes)))
    if work is None or work.numel() < nbytes.value:
        work = torch.empty(nbytes.value, dtype=torch.uint8, device=centroids.device)
    lam_arr = None
    if lam is not None:
        lam_np = np.ascontiguousarray(lam, dtype=np.float64)
        if lam_np.shape != (int(n_parts),):
            raise ValueError("sfc_partition: lam must hold n_parts values")
        lam_arr = lam_np.ctypes.data
    part = torch.empty(n, dtype=torch.int32, device=centroids.device)
    check(load().lesasm_sfc_partition(n, _ptr(centroids), None if weights is None else _ptr(weights), int(n_parts),
                                      lam_arr, int(level), _ptr(work), work.numel(), _ptr(part), _stream()))
    return part


def balance_update(lam_hist, t_hist, growth: float = 1.5) -> np.ndarray:
    """Next correction coefficients (lesasm_balance_update) from the rows of
    coefficients used and part times measured so far."""
    L = np.ascontiguousarray(np.atleast_2d(lam_hist), dtype=np.float64)
    T = np.ascontiguousarray(np.atleast_2d(t_hist), dtype=np.float64)
    if L.shape != T.shape:
        raise ValueError("balance_update: coefficient and time histories differ in shape")
    out = np.empty(L.shape[1], np.float64)
    check(load().lesasm_balance_update(L.shape[1], L.shape[0], L.ctypes.data, T.ctypes.data, float(growth),
                                       out.ctypes.data))
    return out


def _ptrs(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


class Batch:
    """Many meshes assembled by one persistent launch (lesasm_batch_*)."""

    def __init__(self, meshes):
        release_deferred()
        self.meshes = list(meshes)
        arr = (ctypes.c_void_p * len(self.meshes))(*[m._h.value for m in self.meshes])
        h = ctypes.c_void_p()
        check(load().lesasm_batch_create(arr, len(self.meshes), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().lesasm_batch_destroy(self._h)
            self._h = None
        release_deferred()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _defer("lesasm_batch_destroy", h)

    def configure(self, chunk: int = 0, order: int = ORDER_MESH, grid_per_cu: int = 2):
        check(load().lesasm_batch_configure(self._h, int(chunk), int(order), int(grid_per_cu)))

    def set_per_type(self, layout):
        """Kernel layout: 0 / False one persistent kernel for all types, 1 / True
        one persistent kernel per element type, 2 one kernel per element type
        with one workgroup per queue item."""
        check(load().lesasm_batch_set_per_type(self._h, int(layout)))

    def config(self) -> dict:
        c, o, g, n, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(load().lesasm_batch_get_config(self._h, ctypes.byref(c), ctypes.byref(o), ctypes.byref(g), ctypes.byref(n)))
        check(load().lesasm_batch_get_per_type(self._h, ctypes.byref(t)))
        return {"chunk": c.value, "order": o.value, "grid_per_cu": g.value, "items": n.value, "per_type": t.value}

    def _args(self, us, ps, nus):
        nu = (ctypes.c_double * len(nus))(*[float(v) for v in nus])
        return _ptrs(us), (None if ps is None else _ptrs(ps)), nu

    def assemble(self, us, ps, nus, outs=None):
        if outs is None:
            outs = [torch.empty_like(u) for u in us]
        u, p, nu = self._args(us, ps, nus)
        check(load().lesasm_batch_assemble(self._h, u, p, nu, _ptrs(outs), _stream()))
        return outs

    def tune(self, us, ps, nus, outs, cache_path: str | None = None, reps: int = 3) -> float:
        u, p, nu = self._args(us, ps, nus)
        best = ctypes.c_double()
        check(load().lesasm_batch_tune(self._h, u, p, nu, _ptrs(outs),
                                       None if cache_path is None else cache_path.encode(), int(reps),
                                       ctypes.byref(best)))
        return best.value

    def rk3_graph(self, us, ps, nus, dt: float, stream):
        """Capture the three-stage update of all meshes on `stream` (a torch.cuda.Stream)."""
        u, p, nu = self._args(us, ps, nus)
        self._keep = (u, p, nu)
        check(load().lesasm_batch_rk3_graph(self._h, u, p, nu, float(dt), ctypes.c_void_p(stream.cuda_stream)))

    def rk3_launch(self, stream=None):
        s = torch.cuda.current_stream() if stream is None else stream
        check(load().lesasm_batch_rk3_launch(self._h, ctypes.c_void_p(s.cuda_stream)))

    def rk3_eager(self, us, ps, nus, dt: float):
        u, p, nu = self._args(us, ps, nus)
        check(load().lesasm_batch_rk3_eager(self._h, u, p, nu, float(dt), _stream()))


class MLP:
    """The learned subgrid closure network on the GPU (lesasm_mlp_*)."""

    def __init__(self, params: np.ndarray):
        release_deferred()
        p = np.ascontiguousarray(params, np.float32)
        if p.size != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters")
        h = ctypes.c_void_p()
        check(load().lesasm_mlp_create(p.ctypes.data, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().lesasm_mlp_destroy(self._h)
            self._h = None
        release_deferred()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _defer("lesasm_mlp_destroy", h)

    def params(self) -> np.ndarray:
        out = np.empty(MLP_PARAMS, np.float32)
        check(load().lesasm_mlp_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, np.float32)
        check(load().lesasm_mlp_set_params(self._h, p.ctypes.data))

    @staticmethod
    def _f32(t, cols):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 2 and t.shape[1] == cols):
            raise ValueError(f"expected a contiguous float32 [n, {cols}] GPU tensor")
        return t

    def loss_grad(self, x, t):
        self._f32(x, 10), self._f32(t, 6)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        check(load().lesasm_mlp_loss_grad(self._h, _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss), _stream()))
        return loss, g

    def loss_grad_noalloc(self, x, t, grad, loss):
        """loss_grad into caller buffers with no device allocation by the
        library (at most 8192 samples)."""
        self._f32(x, 10), self._f32(t, 6)
        check(load().lesasm_mlp_loss_grad_noalloc(self._h, _ptr(x), _ptr(t), x.shape[0], _ptr(grad), _ptr(loss),
                                                  _stream()))

    def adam(self, grad=None, lr: float = 1e-3):
        check(load().lesasm_mlp_adam(self._h, _ptr(grad), ctypes.c_float(lr), _stream()))

    def train_step(self, x, t, lr: float = 1e-3, loss=None):
        self._f32(x, 10), self._f32(t, 6)
        check(load().lesasm_mlp_train_step(self._h, _ptr(x), _ptr(t), x.shape[0], ctypes.c_float(lr), _ptr(loss),
                                           _stream()))

    def commit(self):
        check(load().lesasm_mlp_commit(self._h))

    def forward_f32(self, x):
        self._f32(x, 10)
        y = torch.empty((x.shape[0], 6), dtype=torch.float32, device=x.device)
        check(load().lesasm_mlp_forward_f32(self._h, _ptr(x), x.shape[0], _ptr(y), _stream()))
        return y

    def infer_bf16(self, x):
        self._f32(x, 10)
        y = torch.empty((x.shape[0], 6), dtype=torch.float32, device=x.device)
        check(load().lesasm_mlp_infer_bf16(self._h, _ptr(x), x.shape[0], _ptr(y), _stream()))
        return y


def set_closure(mesh: Mesh, mlp: "MLP | None", delta_ref: float = 1.0, fallback_tol: float = 0.05):
    check(load().lesasm_mesh_set_closure(mesh._h, None if mlp is None else mlp._h, float(delta_ref),
                                         float(fallback_tol)))
    mesh._closure = mlp  # the mesh uses the network's device weights: keep it alive as long


def closure_fallbacks(mesh: Mesh) -> int:
    v = ctypes.c_uint64()
    check(load().lesasm_mesh_closure_fallbacks(mesh._h, ctypes.byref(v)))
    return v.value


def closure_fallbacks_by_type(mesh: Mesh) -> dict:
    """Elements per type (4, 5, 6, 8) that kept Vreman's stress since the last
    call (resets the counts)."""
    v = (ctypes.c_uint64 * 4)()
    check(load().lesasm_mesh_closure_fallbacks_by_type(mesh._h, v))
    return {4: int(v[0]), 5: int(v[1]), 6: int(v[2]), 8: int(v[3])}
