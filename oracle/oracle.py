"""ctypes wrapper and gcc build of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lesasm_oracle.c")
LIB = os.path.join(HERE, "_build", "liblesasm_oracle.so")

TERM_CONV, TERM_PRES, TERM_VISC, TERM_SGS, TERM_LITERAL = 1, 2, 4, 8, 16
TERM_ALL = TERM_CONV | TERM_PRES | TERM_VISC | TERM_SGS

_lock = threading.Lock()
_lib = None


def build(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle with plain gcc -O2 (no fast-math, no FMA contraction)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
                           "-Wall", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def load():
    """Load the oracle; ``LESASM_ORACLE_LIB`` may name another build of the same
    source (used by the mutation test to run the pins against planted bugs)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = os.environ.get("LESASM_ORACLE_LIB")
        if not path:
            path = LIB
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.oracle_nnode.argtypes = [i32]
        lib.oracle_ngauss.argtypes = [i32]
        lib.oracle_shape.argtypes = [i32, P, P, P]
        lib.oracle_gauss.argtypes = [i32, P, P]
        lib.oracle_vreman.argtypes = [P, f64, f64]
        lib.oracle_vreman.restype = f64
        lib.oracle_element_volume.argtypes = [i32, P, P]
        lib.oracle_element_residual.argtypes = [i32, P, P, P, f64, f64, i32, P, P, P]
        lib.oracle_assemble.argtypes = [i64, P, i64, P, P, P, P, i64, P, P, f64, f64, i32, P]
        lib.oracle_assemble_threads.argtypes = [i64, P, i64, P, P, P, P, i64, P, P, f64, f64, i32, i32, P]
        lib.oracle_lumped_mass.argtypes = [i64, P, i64, P, P, P, P, i64, P]
        lib.oracle_filter_width.argtypes = [i64, P, i64, P, P, P, P]
        lib.oracle_element_laplacian.argtypes = [i32, P, P]
        lib.oracle_divergence.argtypes = [i64, P, i64, P, P, P, P, i64, P, P]
        lib.oracle_element_stress_residual.argtypes = [i32, P, P, P]
        lib.oracle_wall_law.argtypes = [f64]
        lib.oracle_wall_law.restype = f64
        lib.oracle_friction_velocity.argtypes = [f64, f64, f64]
        lib.oracle_friction_velocity.restype = f64
        lib.oracle_wall_assemble.argtypes = [i64, P, i64, P, P, P, P, i64, P, f64, i64, P, P, P, P, P, P, P]
        lib.oracle_bad_element.restype = ctypes.c_longlong
        _lib = lib
        return lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleError(RuntimeError):
    def __init__(self, code, element):
        super().__init__(f"oracle error {code} at element {element}")
        self.code = code
        self.element = element


def _check(st):
    if st != 0:
        raise OracleError(st, load().oracle_bad_element())


def nnode(t: int) -> int:
    return load().oracle_nnode(t)


def ngauss(t: int) -> int:
    return load().oracle_ngauss(t)


def shape(t: int, xi) -> tuple[np.ndarray, np.ndarray]:
    n = nnode(t)
    xi = _f64(xi, (3,))
    N, dN = np.zeros(n), np.zeros((n, 3))
    _check(load().oracle_shape(t, _p(xi), _p(N), _p(dN)))
    return N, dN


def gauss(t: int) -> tuple[np.ndarray, np.ndarray]:
    g = ngauss(t)
    pts, w = np.zeros((g, 3)), np.zeros(g)
    assert load().oracle_gauss(t, _p(pts), _p(w)) == g
    return pts, w


def vreman(G, delta: float, c: float) -> float:
    G = _f64(G, (3, 3))
    return load().oracle_vreman(_p(G), float(delta), float(c))


def element_volume(t: int, x) -> float:
    x = _f64(x)
    v = ctypes.c_double()
    _check(load().oracle_element_volume(t, _p(x), ctypes.addressof(v)))
    return v.value


def element_residual(t: int, x, u, p=None, nu=0.0, c=0.0, terms=TERM_ALL):
    """Returns (R [n,3], per-Gauss-point records [g,18], Delta_e)."""
    x, u = _f64(x), _f64(u)
    p = None if p is None else _f64(p)
    n, g = nnode(t), ngauss(t)
    R, gp = np.zeros((n, 3)), np.zeros((g, 18))
    d = ctypes.c_double()
    _check(load().oracle_element_residual(t, _p(x), _p(u), _p(p), float(nu), float(c), int(terms),
                                          _p(R), _p(gp), ctypes.addressof(d)))
    return R, gp, d.value


def _mesh_args(mesh):
    coords = _f64(mesh.coords)
    types = np.ascontiguousarray(mesh.types, dtype=np.uint8)
    offs = np.ascontiguousarray(mesh.conn_offsets, dtype=np.int64)
    conn = np.ascontiguousarray(mesh.conn, dtype=np.int32)
    fn = None if mesh.field_node is None else np.ascontiguousarray(mesh.field_node, dtype=np.int32)
    nf = mesh.n_field_nodes if fn is not None else len(coords)
    return coords, types, offs, conn, fn, nf


def assemble(mesh, u, p=None, nu=0.0, c=0.1, terms=TERM_ALL) -> np.ndarray:
    """Nodal right-hand side [n_field_nodes, 3] of M_L du/dt = rhs."""
    coords, types, offs, conn, fn, nf = _mesh_args(mesh)
    u = _f64(u, (nf, 3))
    p = None if p is None else _f64(p, (nf,))
    rhs = np.zeros((nf, 3))
    _check(load().oracle_assemble(len(coords), _p(coords), len(types), _p(types), _p(offs), _p(conn), _p(fn), nf,
                                  _p(u), _p(p), float(nu), float(c), int(terms), _p(rhs)))
    return rhs


def assemble_threads(mesh, u, p=None, nu=0.0, c=0.1, threads=1, terms=TERM_ALL) -> np.ndarray:
    """The same assembly split over `threads` OpenMP threads (contiguous element
    ranges, private right-hand sides summed in thread order): the timing leg of
    the benchmark's CPU baseline.  Equal to assemble() up to the order of the
    nodal sums."""
    coords, types, offs, conn, fn, nf = _mesh_args(mesh)
    u = _f64(u, (nf, 3))
    p = None if p is None else _f64(p, (nf,))
    rhs = np.zeros((nf, 3))
    _check(load().oracle_assemble_threads(len(coords), _p(coords), len(types), _p(types), _p(offs), _p(conn), _p(fn),
                                          nf, _p(u), _p(p), float(nu), float(c), int(terms), int(threads), _p(rhs)))
    return rhs


def lumped_mass(mesh) -> np.ndarray:
    coords, types, offs, conn, fn, nf = _mesh_args(mesh)
    M = np.zeros(nf)
    _check(load().oracle_lumped_mass(len(coords), _p(coords), len(types), _p(types), _p(offs), _p(conn), _p(fn),
                                     nf, _p(M)))
    return M


def filter_width(mesh) -> np.ndarray:
    coords, types, offs, conn, _, _ = _mesh_args(mesh)
    d = np.zeros(len(types))
    _check(load().oracle_filter_width(len(coords), _p(coords), len(types), _p(types), _p(offs), _p(conn), _p(d)))
    return d


def element_laplacian(t: int, x) -> np.ndarray:
    x = _f64(x)
    n = nnode(t)
    K = np.zeros((n, n))
    _check(load().oracle_element_laplacian(t, _p(x), _p(K)))
    return K


def divergence(mesh, u) -> np.ndarray:
    """(D u)_a = sum over elements of int N_a div u, [n_field_nodes]."""
    coords, types, offs, conn, fn, nf = _mesh_args(mesh)
    u = _f64(u, (nf, 3))
    out = np.zeros(nf)
    _check(load().oracle_divergence(len(coords), _p(coords), len(types), _p(types), _p(offs), _p(conn), _p(fn), nf,
                                    _p(u), _p(out)))
    return out


def element_stress_residual(t: int, x, tau) -> np.ndarray:
    """R[a, i] = int dN_a/dx_j tau_ij dV for tau given per Gauss point [g, 6]."""
    x = _f64(x)
    tau = _f64(tau, (ngauss(t), 6))
    R = np.zeros((nnode(t), 3))
    _check(load().oracle_element_stress_residual(t, _p(x), _p(tau), _p(R)))
    return R


def wall_law(yp: float) -> float:
    """Reichardt's law of the wall, u+ as a function of y+."""
    return load().oracle_wall_law(float(yp))


def friction_velocity(U: float, y: float, nu: float) -> float:
    """u_tau solving U = u_tau f(y u_tau / nu)."""
    return load().oracle_friction_velocity(float(U), float(y), float(nu))


def wall_assemble(mesh, u, nu: float, face_offsets, face_conn, face_elem):
    """Wall-model nodal contributions [n_field_nodes, 3] (boundary assembly)
    and per-face diagnostics (y, U, u_tau)."""
    coords, types, offs, conn, fn, nf = _mesh_args(mesh)
    u = _f64(u, (nf, 3))
    fo = np.ascontiguousarray(face_offsets, dtype=np.int64)
    fc = np.ascontiguousarray(face_conn, dtype=np.int32)
    fe = np.ascontiguousarray(face_elem, dtype=np.int64)
    nfaces = len(fe)
    out = np.zeros((nf, 3))
    y, U, ut = np.zeros(nfaces), np.zeros(nfaces), np.zeros(nfaces)
    _check(load().oracle_wall_assemble(len(coords), _p(coords), len(types), _p(types), _p(offs), _p(conn), _p(fn), nf,
                                       _p(u), float(nu), nfaces, _p(fo), _p(fc), _p(fe), _p(out), _p(y), _p(U),
                                       _p(ut)))
    return out, y, U, ut
