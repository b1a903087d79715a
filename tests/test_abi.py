"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function that include/lesasm.h declares,
and reject invalid mesh descriptions during validation, before any HIP call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lesasm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lesasm_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2005_05899_amd import lesasm
    if not os.path.exists(lesasm.LIB_PATH):
        pytest.skip("library not built")
    return lesasm.load()


def test_header_declares_the_binding_exports():
    from paper_2005_05899_amd import lesasm
    assert declared_functions() == sorted(lesasm.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_error_text(lib):
    assert lib.lesasm_version() == 1
    assert isinstance(lib.lesasm_last_error(), bytes)


def _desc(lesasm, coords, types, offs, conn, fmap=None, nf=0, c=0.1, flags=0):
    keep = [np.ascontiguousarray(a) for a in (coords, types, offs, conn)]
    d = lesasm.MeshDesc(len(keep[0]), keep[0].ctypes.data, len(keep[1]), keep[1].ctypes.data, keep[2].ctypes.data,
                        keep[3].ctypes.data, None if fmap is None else fmap.ctypes.data, nf, c, flags)
    return d, keep


def _create(lesasm, d):
    h = ctypes.c_void_p()
    st = lesasm.load().lesasm_mesh_create(ctypes.byref(d), ctypes.byref(h))
    return st, h


def test_invalid_descriptions_are_rejected_before_any_gpu_call(lib):
    from paper_2005_05899_amd import lesasm, meshgen
    m = meshgen.uniform_hex_box((2, 1, 1))
    ok = (m.coords, m.types, m.conn_offsets, m.conn)
    # bad type code
    d, k = _desc(lesasm, m.coords, np.array([8, 7], np.uint8), m.conn_offsets, m.conn)
    st, h = _create(lesasm, d)
    assert st == lesasm.E_INVALID_ARG and not h.value and b"type 7" in lib.lesasm_last_error()
    # out-of-range node
    bad = m.conn.copy()
    bad[5] = m.n_nodes
    d, k = _desc(lesasm, m.coords, m.types, m.conn_offsets, bad)
    st, h = _create(lesasm, d)
    assert st == lesasm.E_INVALID_ARG and b"references node" in lib.lesasm_last_error()
    # node count does not match the type
    d, k = _desc(lesasm, m.coords, np.array([4, 8], np.uint8), m.conn_offsets, m.conn)
    assert _create(lesasm, d)[0] == lesasm.E_INVALID_ARG
    # bad field map
    fmap = np.zeros(m.n_nodes, np.int32)
    fmap[3] = 9
    d, k = _desc(lesasm, *ok, fmap=fmap, nf=4)
    assert _create(lesasm, d)[0] == lesasm.E_INVALID_ARG
    # negative Vreman constant, unknown flags
    d, k = _desc(lesasm, *ok, c=-1.0)
    assert _create(lesasm, d)[0] == lesasm.E_INVALID_ARG
    d, k = _desc(lesasm, *ok, flags=0x80)
    assert _create(lesasm, d)[0] == lesasm.E_INVALID_ARG
    # NULL arguments
    assert lib.lesasm_mesh_create(None, None) == lesasm.E_INVALID_ARG
    h = ctypes.c_void_p()
    assert lib.lesasm_mesh_create(None, ctypes.byref(h)) == lesasm.E_INVALID_ARG
    assert lib.lesasm_assemble_momentum_rhs(None, None, None, 0.0, 0.0, None, None) == lesasm.E_INVALID_ARG
    assert lib.lesasm_mesh_destroy(None) == lesasm.OK


def test_memory_cap_and_count_without_gpu(lib):
    # host-side bookkeeping: nothing allocated yet in this process, the cap is
    # set and cleared without a GPU
    import ctypes as C
    v = C.c_uint64(123)
    assert lib.lesasm_memory_in_use(C.byref(v)) == 0 and v.value == 0
    assert lib.lesasm_set_memory_cap(1 << 20) == 0
    assert lib.lesasm_set_memory_cap(0) == 0
    assert lib.lesasm_memory_in_use(None) == -1
