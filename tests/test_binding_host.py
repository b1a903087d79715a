"""Host logic of the Python binding, on the CPU (no library call reaches a
GPU): objects dropped by the garbage collector are not destroyed from the
collector (a destroy synchronises the device, which must not happen inside a
caller's stream capture) but at the next explicit release, in dependency
order; a mesh keeps its closure network alive."""
import gc

from paper_2005_05899_amd import lesasm


class _Recorder:
    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        return lambda *args: self.calls.append((name,) + args) or 0


def _bare(cls, h):
    obj = cls.__new__(cls)
    obj._h = h
    return obj


def test_collected_objects_are_destroyed_later_in_dependency_order(monkeypatch):
    rec = _Recorder()
    monkeypatch.setattr(lesasm, "load", lambda *a, **k: rec)
    lesasm._deferred.clear()
    objs = [_bare(lesasm.MLP, 1), _bare(lesasm.Mesh, 2), _bare(lesasm.Stepper, 3), _bare(lesasm.Batch, 4),
            _bare(lesasm.StepGraph, 5), _bare(lesasm.Mesh, 6)]
    del objs
    gc.collect()
    assert rec.calls == []  # nothing destroyed from the collector
    assert len(lesasm._deferred) == 6
    lesasm.release_deferred()
    assert [c[0] for c in rec.calls] == ["lesasm_step_graph_destroy", "lesasm_stepper_destroy",
                                         "lesasm_batch_destroy", "lesasm_mesh_destroy", "lesasm_mesh_destroy",
                                         "lesasm_mlp_destroy"]
    handles = [c[1] for c in rec.calls]
    assert handles[:3] == [5, 3, 4] and sorted(handles[3:5]) == [2, 6] and handles[5] == 1
    assert lesasm._deferred == []
    lesasm.release_deferred()  # nothing left: no further calls
    assert len(rec.calls) == 6


def test_explicit_close_destroys_at_once_and_releases_the_queue(monkeypatch):
    rec = _Recorder()
    monkeypatch.setattr(lesasm, "load", lambda *a, **k: rec)
    lesasm._deferred.clear()
    dropped = _bare(lesasm.Mesh, 7)
    del dropped
    gc.collect()
    m = _bare(lesasm.Mesh, 8)
    m.close()
    assert [c[:2] for c in rec.calls] == [("lesasm_mesh_destroy", 8), ("lesasm_mesh_destroy", 7)]
    m.close()  # closing twice is a no-op
    assert len(rec.calls) == 2


def test_mesh_keeps_its_closure_network(monkeypatch):
    rec = _Recorder()
    monkeypatch.setattr(lesasm, "load", lambda *a, **k: rec)
    monkeypatch.setattr(lesasm, "check", lambda status: None)
    lesasm._deferred.clear()
    m = _bare(lesasm.Mesh, 9)
    net = _bare(lesasm.MLP, 10)
    lesasm.set_closure(m, net, 0.1, 0.05)
    del net
    gc.collect()
    assert lesasm._deferred == []  # still referenced by the mesh
    lesasm.set_closure(m, None)
    gc.collect()
    assert [d[2:] for d in lesasm._deferred] == [("lesasm_mlp_destroy", 10)]
    lesasm._deferred.clear()
    m._h = None
