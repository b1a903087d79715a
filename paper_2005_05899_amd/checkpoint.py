"""Checkpoint and resume of a simulation state: velocity u [n,3], pressure
p [n] (user node order), step count, time and the seeds of the run, tied to
the mesh they belong to.

Files are numpy .npz archives of plain arrays (no pickled objects; loading
uses allow_pickle=False).  A state records a signature of the mesh (element
types, connectivity, periodic map, node counts) and is refused for another
mesh.  The device side converts between the mesh's internal order and the
user order (save_device / load_device)."""
from __future__ import annotations

import hashlib
import json

import numpy as np

FORMAT = "lesasm-state-1"


def mesh_signature(mesh) -> str:
    """SHA-256 over the mesh's node counts, element types, connectivity and
    periodic map (any object with the meshgen.Mesh fields)."""
    h = hashlib.sha256()
    h.update(np.asarray([len(mesh.coords), len(mesh.types), int(getattr(mesh, "n_field_nodes", 0) or 0)],
                        np.int64).tobytes())
    for a in (mesh.types, mesh.conn_offsets, mesh.conn):
        h.update(np.ascontiguousarray(a).tobytes())
    fn = getattr(mesh, "field_node", None)
    h.update(b"periodic" if fn is not None else b"plain")
    if fn is not None:
        h.update(np.ascontiguousarray(fn, np.int32).tobytes())
    return h.hexdigest()


def save(path: str, mesh, u: np.ndarray, p: np.ndarray, step: int, t: float, seeds: dict | None = None) -> None:
    """Write the state (host arrays in user node order)."""
    u = np.ascontiguousarray(u, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    n = u.shape[0]
    if u.ndim != 2 or u.shape[1] != 3 or p.shape != (n,):
        raise ValueError("checkpoint: u must be [n, 3] and p [n]")
    meta = {"format": FORMAT, "step": int(step), "t": float(t), "seeds": seeds or {},
            "mesh": mesh_signature(mesh), "n": int(n)}
    with open(path, "wb") as f:
        np.savez(f, u=u, p=p, meta=np.frombuffer(json.dumps(meta).encode(), np.uint8))


def load(path: str, mesh):
    """Read a state written by save() for this mesh.  Returns (u, p, step, t,
    seeds); raises ValueError for another format or another mesh."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(z["meta"].tobytes().decode())
        if meta.get("format") != FORMAT:
            raise ValueError(f"checkpoint: unknown format {meta.get('format')!r}")
        if meta["mesh"] != mesh_signature(mesh):
            raise ValueError("checkpoint: the state belongs to another mesh")
        u, p = np.array(z["u"]), np.array(z["p"])
    if u.shape != (meta["n"], 3) or p.shape != (meta["n"],):
        raise ValueError("checkpoint: field sizes do not match the record")
    return u, p, meta["step"], meta["t"], meta["seeds"]


def save_device(path: str, host_mesh, dev_mesh, u, p, step: int, t: float, seeds: dict | None = None) -> None:
    """save() from device tensors in the library mesh's internal order."""
    save(path, host_mesh, dev_mesh.to_user(u).cpu().numpy(), dev_mesh.to_user(p.reshape(-1, 1)).cpu().numpy()[:, 0],
         step, t, seeds)


def load_device(path: str, host_mesh, dev_mesh):
    """load() into device tensors in the library mesh's internal order."""
    import torch
    u, p, step, t, seeds = load(path, host_mesh)
    ud = dev_mesh.to_internal(torch.from_numpy(u).to(dev_mesh.device))
    pd = dev_mesh.to_internal(torch.from_numpy(p).to(dev_mesh.device))
    return ud, pd, step, t, seeds
