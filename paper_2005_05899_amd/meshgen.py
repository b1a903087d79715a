"""Seeded synthetic workloads for the LES momentum-residual assembly.

This module only builds inputs: node coordinates, element connectivity and
nodal fields.  It holds no part of the assembly itself (no shape functions,
quadrature, Jacobians, filter widths or masses), so both the CPU oracle and the
GPU path can be fed from it without sharing any of the method's arithmetic.

Element types follow the paper's hybrid linear meshes (Section 3.3: tetrahedra,
prisms, pyramids; hexahedra for the periodic cube):

* ``TET04`` nodes: reference (0,0,0), (1,0,0), (0,1,0), (0,0,1).
* ``PYR05`` nodes: base (-1,-1,0), (1,-1,0), (1,1,0), (-1,1,0), apex (0,0,1).
* ``PEN06`` nodes: triangle (0,0), (1,0), (0,1) at zeta=-1, then the same at +1.
* ``HEX08`` nodes: (-1,-1,-1), (1,-1,-1), (1,1,-1), (-1,1,-1), then zeta=+1.

Every generator is deterministic in its seed (numpy PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from itertools import permutations

import numpy as np

TET04, PYR05, PEN06, HEX08 = 4, 5, 6, 8
NNODE = {TET04: 4, PYR05: 5, PEN06: 6, HEX08: 8}
TYPE_NAME = {TET04: "TET04", PYR05: "PYR05", PEN06: "PEN06", HEX08: "HEX08"}


@dataclass
class Mesh:
    """A linear hybrid mesh in plain arrays.

    ``coords``       float64 [n_nodes, 3]  geometry node coordinates
    ``types``        uint8   [n_elems]     4, 5, 6 or 8
    ``conn_offsets`` int64   [n_elems + 1] CSR offsets into ``conn``
    ``conn``         int32   [nnz]         geometry node ids per element
    ``field_node``   int32   [n_nodes] or None: field (unknown) node of each
                     geometry node; periodic copies share one field node
    ``n_field_nodes``                      number of field nodes
    """

    coords: np.ndarray
    types: np.ndarray
    conn_offsets: np.ndarray
    conn: np.ndarray
    field_node: np.ndarray | None = None
    n_field_nodes: int = 0
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.n_field_nodes == 0:
            self.n_field_nodes = (int(self.field_node.max()) + 1
                                  if self.field_node is not None else len(self.coords))

    @property
    def n_nodes(self) -> int:
        return len(self.coords)

    @property
    def n_elems(self) -> int:
        return len(self.types)

    def field_coords(self) -> np.ndarray:
        """Coordinates of each field node (first geometry node mapped to it)."""
        if self.field_node is None:
            return self.coords
        out = np.empty((self.n_field_nodes, 3))
        # reversed so that the lowest geometry id wins
        out[self.field_node[::-1]] = self.coords[::-1]
        return out

    def type_counts(self) -> dict:
        return {TYPE_NAME[t]: int((self.types == t).sum()) for t in (TET04, PYR05, PEN06, HEX08)}

    def element_nodes(self, e: int) -> np.ndarray:
        return self.conn[self.conn_offsets[e]:self.conn_offsets[e + 1]]


def _csr(types: np.ndarray, blocks: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    lut = np.zeros(9, np.int64)
    for t, n in NNODE.items():
        lut[t] = n
    counts = lut[types]
    offsets = np.zeros(len(types) + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    conn = np.concatenate([b.reshape(-1) for b in blocks]).astype(np.int32) if blocks else np.zeros(0, np.int32)
    assert len(conn) == offsets[-1]
    return offsets, conn


# ---------------------------------------------------------------------------
# Periodic uniform HEX08 cube
# ---------------------------------------------------------------------------

_HEX_CORNERS = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]


def periodic_hex_cube(n: int = 16, length: float = 2.0 * math.pi) -> Mesh:
    """n^3 uniform HEX08 cells on [0, L]^3; (n+1)^3 geometry nodes, n^3 field nodes."""
    m = n + 1
    h = length / n
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    coords = np.stack([i * h, j * h, k * h], axis=1).astype(np.float64)
    field_node = ((i % n) + n * ((j % n) + n * (k % n))).astype(np.int32)
    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    cols = [(ci + dx) + m * ((cj + dy) + m * (ck + dz)) for dx, dy, dz in _HEX_CORNERS]
    conn_e = np.stack(cols, axis=1)
    types = np.full(n ** 3, HEX08, np.uint8)
    offsets, conn = _csr(types, [conn_e])
    return Mesh(coords, types, offsets, conn, field_node, n ** 3,
                meta={"kind": "periodic_hex_cube", "n": n, "length": length})


def uniform_hex_box(n: tuple[int, int, int], length=(1.0, 1.0, 1.0)) -> Mesh:
    """Non-periodic uniform HEX08 grid on [0, Lx] x [0, Ly] x [0, Lz]."""
    nx, ny, nz = n
    hx, hy, hz = (length[0] / nx, length[1] / ny, length[2] / nz)
    mx, my, mz = nx + 1, ny + 1, nz + 1
    k, j, i = np.meshgrid(np.arange(mz), np.arange(my), np.arange(mx), indexing="ij")
    coords = np.stack([i.ravel() * hx, j.ravel() * hy, k.ravel() * hz], axis=1).astype(np.float64)
    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    cols = [(ci + dx) + mx * ((cj + dy) + my * (ck + dz)) for dx, dy, dz in _HEX_CORNERS]
    types = np.full(nx * ny * nz, HEX08, np.uint8)
    offsets, conn = _csr(types, [np.stack(cols, axis=1)])
    return Mesh(coords, types, offsets, conn, None, 0, meta={"kind": "uniform_hex_box", "n": n})


# ---------------------------------------------------------------------------
# Graded, perturbed, z-layered hybrid box
# ---------------------------------------------------------------------------

def _signed_volume(a, b, c, d) -> float:
    return float(np.dot(np.subtract(b, a), np.cross(np.subtract(c, a), np.subtract(d, a))) / 6.0)


def _split_templates() -> dict:
    """Per-type splits of a unit cell into elements, as corner codes.

    A code is a (dx, dy, dz) corner or the string "c" (cell centre, pyramids).
    Orientation is fixed on the unit cube so that every element has a positive
    signed volume in the node order listed in the module docstring.
    """
    cube = {c: np.array(c, float) for c in _HEX_CORNERS}
    centre = np.array([0.5, 0.5, 0.5])

    def pos(code):
        return centre if code == "c" else cube[code]

    # Kuhn split: six monotone corner paths from (0,0,0) to (1,1,1); every
    # cube face is cut along the diagonal through its lowest corner, which is
    # the diagonal the prism split below uses on the horizontal faces.
    tets = []
    for perm in permutations(range(3)):
        v = [np.zeros(3, int)]
        for ax in perm:
            step = v[-1].copy()
            step[ax] += 1
            v.append(step)
        codes = [tuple(int(t) for t in p) for p in v]
        if _signed_volume(*[pos(c) for c in codes]) < 0:
            codes[1], codes[2] = codes[2], codes[1]
        tets.append(codes)

    # Two prisms cut by the (0,0)-(1,1) diagonal of the horizontal faces.
    pens = [
        [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1)],
        [(0, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1), (0, 1, 1)],
    ]
    for p in pens:
        assert _signed_volume(pos(p[0]), pos(p[1]), pos(p[2]), pos(p[3])) > 0

    # Six pyramids, one per cube face, apex at the cell centre.
    faces = [
        [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0)],
        [(0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)],
        [(0, 0, 0), (1, 0, 0), (1, 0, 1), (0, 0, 1)],
        [(0, 1, 0), (1, 1, 0), (1, 1, 1), (0, 1, 1)],
        [(0, 0, 0), (0, 1, 0), (0, 1, 1), (0, 0, 1)],
        [(1, 0, 0), (1, 1, 0), (1, 1, 1), (1, 0, 1)],
    ]
    pyrs = []
    for f in faces:
        if _signed_volume(pos(f[0]), pos(f[1]), pos(f[2]), centre) < 0:
            f = [f[0], f[3], f[2], f[1]]
        pyrs.append(f + ["c"])
    hexes = [list(_HEX_CORNERS)]
    return {TET04: tets, PEN06: pens, PYR05: pyrs, HEX08: hexes}


SPLITS = _split_templates()
ELEMS_PER_CELL = {t: len(v) for t, v in SPLITS.items()}


def graded_spacing(nz: int, length: float, ratio: float = 1.2, n_graded: int = 10) -> np.ndarray:
    """Layer heights growing geometrically by ``ratio`` from z=0 for ``n_graded``
    layers, then constant (the core spacing), scaled to total ``length``."""
    rel = np.minimum(1.0, ratio ** (np.arange(nz, dtype=float) - n_graded))
    return rel * (length / rel.sum())


def hybrid_box(nx: int, ny: int, layers, length=(2 * math.pi,) * 3, ratio: float = 1.2,
               n_graded: int = 10, perturb: float = 0.1, seed: int = 0) -> Mesh:
    """Hybrid box built from a z-graded, randomly perturbed hex grid.

    ``layers`` lists (type, number of cell layers) from the wall z=0 upward.
    Each cell of a layer is split into that type (6 TET04, 2 PEN06, 6 PYR05
    around a centre node, or 1 HEX08), so type changes happen on whole planes.
    Interior nodes move by U(-perturb, perturb) times the local spacing in each
    component; boundary nodes keep the coordinate of their boundary plane.
    """
    rng = np.random.default_rng(seed)
    nz = int(sum(n for _, n in layers))
    lx, ly, lz = length
    hx, hy = lx / nx, ly / ny
    dz = graded_spacing(nz, lz, ratio, n_graded) if nz else np.zeros(0)
    zs = np.concatenate([[0.0], np.cumsum(dz)])
    zs[-1] = lz
    mx, my, mz = nx + 1, ny + 1, nz + 1
    k, j, i = np.meshgrid(np.arange(mz), np.arange(my), np.arange(mx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    coords = np.stack([i * hx, j * hy, zs[k]], axis=1)
    # local spacing for the perturbation (min of the two adjacent layers in z)
    dz_ext = np.concatenate([[dz[0] if nz else 0.0], dz, [dz[-1] if nz else 0.0]])
    hz_loc = np.minimum(dz_ext[k], dz_ext[k + 1])
    noise = rng.uniform(-perturb, perturb, size=(len(coords), 3))
    noise[:, 0] *= hx * ((i > 0) & (i < nx))
    noise[:, 1] *= hy * ((j > 0) & (j < ny))
    noise[:, 2] *= hz_loc * ((k > 0) & (k < nz))
    coords = coords + noise
    n_grid = len(coords)

    type_blocks, conn_blocks, centre_coords = [], [], []
    next_centre = n_grid
    k0 = 0
    layer_info = []
    for t, nl in layers:
        if nl == 0:
            continue
        ck, cj, ci = np.meshgrid(np.arange(k0, k0 + nl), np.arange(ny), np.arange(nx), indexing="ij")
        ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
        ncell = len(ci)
        corner = {c: (ci + c[0]) + mx * ((cj + c[1]) + my * (ck + c[2])) for c in _HEX_CORNERS}
        if t == PYR05:
            centre = np.arange(next_centre, next_centre + ncell)
            next_centre += ncell
            pts = np.stack([coords[corner[c]] for c in _HEX_CORNERS], axis=0)
            centre_coords.append(pts.mean(axis=0))
        else:
            centre = None
        per_cell = []
        for tmpl in SPLITS[t]:
            per_cell.append(np.stack([centre if c == "c" else corner[c] for c in tmpl], axis=1))
        # element order: cell-major, split index minor
        conn_t = np.stack(per_cell, axis=1).reshape(ncell * len(per_cell), NNODE[t])
        conn_blocks.append(conn_t)
        type_blocks.append(np.full(len(conn_t), t, np.uint8))
        layer_info.append((TYPE_NAME[t], k0, k0 + nl, len(conn_t)))
        k0 += nl
    if centre_coords:
        coords = np.concatenate([coords] + centre_coords, axis=0)
    types = np.concatenate(type_blocks) if type_blocks else np.zeros(0, np.uint8)
    offsets, conn = _csr(types, conn_blocks)
    return Mesh(np.ascontiguousarray(coords, dtype=np.float64), types, offsets, conn, None, 0,
                meta={"kind": "hybrid_box", "nx": nx, "ny": ny, "layers": [(TYPE_NAME[t], n) for t, n in layers],
                      "ratio": ratio, "n_graded": n_graded, "perturb": perturb, "seed": seed,
                      "layer_info": layer_info})


# Faces of each element type as cycles of local nodes (topology only).
FACES = {
    TET04: [(0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)],
    PYR05: [(0, 1, 2, 3), (0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)],
    PEN06: [(0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)],
    HEX08: [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)],
}


def wall_faces(mesh: Mesh, axis: int = 2, value: float = 0.0):
    """Element faces whose nodes all lie on the plane x[axis] == value (the
    generators keep boundary nodes exactly on their plane).  Returns
    (face_offsets int64 [F+1], face_conn int32, face_elem int64 [F]), faces in
    element order, nodes as a cycle of the element's face."""
    on = mesh.coords[:, axis] == value
    elems, conns = [], []
    for t, faces in FACES.items():
        idx = np.where(mesh.types == t)[0]
        if len(idx) == 0:
            continue
        en = mesh.conn[mesh.conn_offsets[idx][:, None] + np.arange(t)[None, :]]
        for f in faces:
            hit = on[en[:, list(f)]].all(axis=1)
            for e, nodes in zip(idx[hit], en[hit][:, list(f)]):
                elems.append(int(e))
                conns.append(nodes)
    order = np.argsort(np.asarray(elems, dtype=np.int64), kind="stable")
    elems = np.asarray(elems, dtype=np.int64)[order]
    conns = [conns[i] for i in order]
    offs = np.zeros(len(conns) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(c) for c in conns])
    flat = np.concatenate(conns).astype(np.int32) if conns else np.zeros(0, np.int32)
    return offs, flat, elems


def hybrid_layers(n_cells_xy: int, target_elems: int, fractions=None) -> list:
    """Whole cell layers per type (wall first: PEN06, TET04, PYR05, HEX08) whose
    element counts come closest to ``fractions`` of ``target_elems``."""
    if fractions is None:
        fractions = {PEN06: 0.40, TET04: 0.40, PYR05: 0.05, HEX08: 0.15}
    out = []
    for t in (PEN06, TET04, PYR05, HEX08):
        nl = max(1, int(round(fractions[t] * target_elems / (ELEMS_PER_CELL[t] * n_cells_xy))))
        out.append((t, nl))
    return out


# ---------------------------------------------------------------------------
# Fields
# ---------------------------------------------------------------------------

def taylor_green_velocity(x: np.ndarray, u0: float = 1.0) -> np.ndarray:
    """u = U0 (sin x cos y cos z, -cos x sin y cos z, 0)."""
    sx, cx = np.sin(x[:, 0]), np.cos(x[:, 0])
    sy, cy = np.sin(x[:, 1]), np.cos(x[:, 1])
    cz = np.cos(x[:, 2])
    return u0 * np.stack([sx * cy * cz, -cx * sy * cz, np.zeros_like(cz)], axis=1)


def taylor_green_pressure(x: np.ndarray, u0: float = 1.0) -> np.ndarray:
    """Kinematic Taylor-Green pressure (U0^2/16)(cos 2x + cos 2y)(cos 2z + 2)."""
    return (u0 ** 2 / 16.0) * (np.cos(2 * x[:, 0]) + np.cos(2 * x[:, 1])) * (np.cos(2 * x[:, 2]) + 2.0)


def taylor_green_modified_pressure(x: np.ndarray, u0: float = 1.0) -> np.ndarray:
    """Pressure with the kinetic energy folded in: p_TG - |u_TG|^2 / 2."""
    u = taylor_green_velocity(x, u0)
    return taylor_green_pressure(x, u0) - 0.5 * (u * u).sum(axis=1)


def _integer_modes(n_modes: int, kmax: int, rng) -> np.ndarray:
    r = np.arange(-kmax, kmax + 1)
    kk = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    k2 = (kk * kk).sum(axis=1)
    keep = (k2 >= 1) & (k2 <= kmax * kmax)
    # one representative of each +-k pair so that no two modes are correlated
    canon = (kk[:, 0] > 0) | ((kk[:, 0] == 0) & (kk[:, 1] > 0)) | ((kk[:, 0] == 0) & (kk[:, 1] == 0) & (kk[:, 2] > 0))
    cand = kk[keep & canon]
    n_modes = min(n_modes, len(cand))
    return cand[rng.choice(len(cand), n_modes, replace=False)].astype(np.float64)


def submesh(mesh: Mesh, elems) -> tuple[Mesh, np.ndarray]:
    """Elements ``elems`` (parent ids, ascending) as a mesh of their own: the
    nodes they use renumbered in ascending parent order (a node on the
    interface with other parts appears in each of them), and, per field node
    of the part, the parent's field node id (to slice field arrays)."""
    elems = np.asarray(elems, np.int64)
    off = mesh.conn_offsets
    cnt = off[elems + 1] - off[elems]
    new_off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    idx = np.repeat(off[elems], cnt) + (np.arange(new_off[-1]) - np.repeat(new_off[:-1], cnt))
    nodes, inv = np.unique(mesh.conn[idx], return_inverse=True)
    types = mesh.types[elems]
    if mesh.field_node is None:
        return Mesh(mesh.coords[nodes], types, new_off, inv.astype(np.int32)), nodes
    fids, finv = np.unique(mesh.field_node[nodes], return_inverse=True)
    return Mesh(mesh.coords[nodes], types, new_off, inv.astype(np.int32), finv.astype(np.int32), len(fids)), fids


@dataclass
class FourierField:
    """u(x) = sum_m a_m cos(k_m . x + phi_m) with integer wave vectors k_m."""

    k: np.ndarray      # [M, 3]
    a: np.ndarray      # [M, ncomp]
    phase: np.ndarray  # [M]

    def __call__(self, x: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
        out = np.empty((len(x), self.a.shape[1]))
        try:  # torch's CPU cos is vectorised and threaded; numpy's is scalar
            import torch
            k, a, ph = (torch.from_numpy(np.ascontiguousarray(v)) for v in (self.k.T, self.a, self.phase))
            for s in range(0, len(x), chunk):
                th = torch.from_numpy(np.ascontiguousarray(x[s:s + chunk])) @ k + ph
                out[s:s + chunk] = (torch.cos(th) @ a).numpy()
        except ImportError:
            for s in range(0, len(x), chunk):
                th = x[s:s + chunk] @ self.k.T + self.phase
                out[s:s + chunk] = np.cos(th) @ self.a
        return out


def random_fourier_velocity(n_modes: int = 512, kmax: int = 16, urms: float = 1.0, seed: int = 3,
                            slope: float = -11.0 / 6.0) -> FourierField:
    """Divergence-free random Fourier field: M integer modes uniform in the ball
    1 <= |k| <= kmax, amplitude |k|^slope, direction a_m perpendicular to k_m,
    uniform random phases, scaled so that sqrt(<|u|^2>/3) = urms."""
    rng = np.random.default_rng(seed)
    k = _integer_modes(n_modes, kmax, rng)
    kn = np.linalg.norm(k, axis=1)
    g = rng.standard_normal(k.shape)
    d = g - ((g * k).sum(axis=1) / kn ** 2)[:, None] * k
    d /= np.linalg.norm(d, axis=1)[:, None]
    a = d * (kn ** slope)[:, None]
    phase = rng.uniform(0.0, 2 * math.pi, len(k))
    mean_sq = 0.5 * (a * a).sum()  # spatial mean of |u|^2 over the periodic box
    a *= urms / math.sqrt(mean_sq / 3.0)
    return FourierField(k, a, phase)


def random_fourier_velocity_peaked(kpeak: float = 4.0, kmax: int = 10, n_modes: int = 512, urms: float = 1.0,
                                   seed: int = 7) -> FourierField:
    """Divergence-free random Fourier field whose shell energy peaks near
    kpeak: mode amplitudes |k| (|k|/kpeak)^2 exp(-(|k|/kpeak)^2) / |k|^2 over
    integer modes uniform in the ball 1 <= |k| <= kmax (initial condition of
    the decaying-turbulence runs)."""
    rng = np.random.default_rng(seed)
    k = _integer_modes(n_modes, kmax, rng)
    kn = np.linalg.norm(k, axis=1)
    g = rng.standard_normal(k.shape)
    d = g - ((g * k).sum(axis=1) / kn ** 2)[:, None] * k
    d /= np.linalg.norm(d, axis=1)[:, None]
    amp = (kn / kpeak) ** 2 * np.exp(-(kn / kpeak) ** 2) / kn
    a = d * amp[:, None]
    phase = rng.uniform(0.0, 2 * math.pi, len(k))
    a *= urms / math.sqrt(0.5 * (a * a).sum() / 3.0)
    return FourierField(k, a, phase)


def random_fourier_scalar(n_modes: int = 128, kmax: int = 8, rms: float = 0.5, seed: int = 11,
                          slope: float = -11.0 / 6.0) -> FourierField:
    """Smooth seeded scalar field (used as a pressure input), rms value ``rms``."""
    rng = np.random.default_rng(seed)
    k = _integer_modes(n_modes, kmax, rng)
    kn = np.linalg.norm(k, axis=1)
    a = (kn ** slope)[:, None] * rng.choice([-1.0, 1.0], size=(len(k), 1))
    phase = rng.uniform(0.0, 2 * math.pi, len(k))
    a *= rms / math.sqrt(0.5 * (a * a).sum())
    return FourierField(k, a, phase)


def uniform_noise(shape, amplitude: float, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-amplitude, amplitude, size=shape)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclass
class Case:
    """A mesh plus the per-call inputs of one momentum-residual assembly."""

    name: str
    mesh: Mesh
    u: np.ndarray            # [n_field_nodes, 3]
    p: np.ndarray | None     # [n_field_nodes]
    nu: float
    vreman_c: float = 0.1
    meta: dict = field(default_factory=dict)


def periodic_tg_case(n: int = 16, noise: float = 1e-3, nu: float = 1e-5, c: float = 0.1, seed: int = 1) -> Case:
    """Periodic cube of n^3 HEX08 on [0, 2 pi]^3 with the Taylor-Green velocity
    plus seeded uniform noise per field node and component, and the modified
    Taylor-Green pressure.  n=16, noise 1e-3, nu 1e-5, c 0.1 is the plain
    CPU-checkable case."""
    mesh = periodic_hex_cube(n)
    xf = mesh.field_coords()
    u = taylor_green_velocity(xf)
    if noise:
        u = u + uniform_noise(u.shape, noise, seed)
    p = taylor_green_modified_pressure(xf)
    return Case(f"periodic_tg_{n}", mesh, u, p, nu, c, meta={"noise": noise, "seed": seed})


def hybrid_case(target_elems: int, seed_mesh: int = 2, seed_u: int = 3, seed_p: int = 11,
                nu: float = 1.5e-5, c: float = 0.1, n_xy: int | None = None, with_p: bool = True,
                n_modes: int = 512) -> Case:
    """Graded, perturbed hybrid box with about ``target_elems`` elements
    (40 % TET04, 40 % PEN06, 5 % PYR05, 15 % HEX08), divergence-free random
    Fourier velocity (512 modes, |k| <= 16, u_rms 1) and a smooth pressure."""
    if n_xy is None:
        # cells per element for the mix: 0.4/6 + 0.4/2 + 0.05/6 + 0.15 -> cube root
        cells = target_elems * (0.4 / 6 + 0.4 / 2 + 0.05 / 6 + 0.15)
        n_xy = max(1, int(round(cells ** (1.0 / 3.0))))
    layers = hybrid_layers(n_xy * n_xy, target_elems)
    mesh = hybrid_box(n_xy, n_xy, layers, seed=seed_mesh)
    xf = mesh.field_coords()
    u = random_fourier_velocity(n_modes=n_modes, seed=seed_u)(xf)
    p = random_fourier_scalar(seed=seed_p)(xf)[:, 0] if with_p else None
    return Case(f"hybrid_{mesh.n_elems}", mesh, u, p, nu, c,
                meta={"seed_mesh": seed_mesh, "seed_u": seed_u, "seed_p": seed_p, "n_xy": n_xy})


def hybrid_2m_case() -> Case:
    """The 2 M-element FP64 GPU workload (95 x 95 cells, 94 layers)."""
    return hybrid_case(2_000_000, seed_mesh=2, seed_u=3, seed_p=11, n_xy=95)


def hybrid_20m_case() -> Case:
    """The 20 M-element hybrid workload (205 x 205 cells), the benchmark's default."""
    return hybrid_case(20_000_000, seed_mesh=4, seed_u=5, seed_p=12, n_xy=205)


def tet_case(n_xy: int = 150, nz: int | None = None, seed_mesh: int = 8, seed_u: int = 9, seed_p: int = 13,
             nu: float = 1.5e-5, c: float = 0.1) -> Case:
    """All-TET04 box: the graded, perturbed hex grid of hybrid_box with every
    cell split into 6 tetrahedra (n_xy = 150: 150 x 150 x 150 cells, 20.25 M
    elements), random Fourier velocity and smooth pressure as hybrid_case."""
    nz = n_xy if nz is None else nz
    mesh = hybrid_box(n_xy, n_xy, [(TET04, nz)], seed=seed_mesh)
    xf = mesh.field_coords()
    u = random_fourier_velocity(seed=seed_u)(xf)
    p = random_fourier_scalar(seed=seed_p)(xf)[:, 0]
    return Case(f"tet_{mesh.n_elems}", mesh, u, p, nu, c,
                meta={"seed_mesh": seed_mesh, "seed_u": seed_u, "seed_p": seed_p, "n_xy": n_xy, "nz": nz})


def small_hybrid_case(nx: int = 5, ny: int = 4, layers=None, seed: int = 7, nu: float = 0.05,
                      c: float = 0.1, with_p: bool = True) -> Case:
    """A few hundred elements of every type (several tiles plus ragged tails)."""
    if layers is None:
        layers = [(PEN06, 2), (TET04, 2), (PYR05, 1), (HEX08, 2)]
    mesh = hybrid_box(nx, ny, layers, seed=seed)
    xf = mesh.field_coords()
    u = random_fourier_velocity(n_modes=64, kmax=4, seed=seed + 100)(xf)
    p = random_fourier_scalar(n_modes=32, kmax=3, seed=seed + 200)(xf)[:, 0] if with_p else None
    return Case(f"small_hybrid_{mesh.n_elems}", mesh, u, p, nu, c, meta={"seed": seed})


def partition_sizes(n_parts: int = 64, lo: float = 5e4, hi: float = 2e6, total: float = 25e6,
                    seed: int = 6) -> np.ndarray:
    """Element counts log-uniform in [lo, hi], rescaled so that they sum to
    about ``total`` (rescaled values clipped back into [lo, hi])."""
    rng = np.random.default_rng(seed)
    e = np.exp(rng.uniform(math.log(lo), math.log(hi), n_parts))
    e *= total / e.sum()
    return np.clip(np.round(e), lo, hi).astype(np.int64)
