"""The C-ABI library loads and exports every entry point the public header
declares; argument checks run on the host before any device work."""
import ctypes
import os
import re

import numpy as np

from paper_2608_27863_amd import hdg, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hdg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hdg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("hdg_local_residual_jacobian", "hdg_condense", "hdg_face_matvec", "hdg_asm_block_apply",
              "hdg_recover_interior"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = hdg.load_library()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(hdg.EXPORTS) <= set(_declared())


def _desc(mesh, keep):
    keep.update(vert=np.ascontiguousarray(mesh.vert_xyz), ev=np.ascontiguousarray(mesh.elem_vert, np.int32),
                ef=np.ascontiguousarray(mesh.elem_face, np.int32), fe=np.ascontiguousarray(mesh.face_elem, np.int32),
                bc=np.ascontiguousarray(mesh.face_bc, np.int8), p=np.ascontiguousarray(mesh.elem_p, np.int8))
    return hdg._MeshDesc(mesh.n_elem, mesh.n_face, mesh.n_vert, *(keep[k].ctypes.data for k in
                                                                  ("vert", "ev", "ef", "fe", "bc", "p")))


def test_create_rejects_inconsistent_meshes_before_touching_the_device():
    L = hdg.load_library()
    phys = hdg._Phys(1.4, 0.71, 1600.0, 0.1, 5.0, 0.01, synth.dirk_alpha(), 1)
    h = ctypes.c_void_p()
    bad_cases = []
    m = synth.box_mesh((2, 2, 2), p=2)
    keep = {}
    d = _desc(m, keep)
    keep["ef"][0, 0] = 10 ** 6             # face index out of range
    bad_cases.append(d)
    keep2 = {}
    d2 = _desc(m, keep2)
    keep2["p"][3] = 5                      # degree outside 1..4
    bad_cases.append(d2)
    keep3 = {}
    d3 = _desc(m, keep3)
    keep3["fe"][0, 1, 1] = keep3["fe"][0, 0, 1]  # both sides on the same local face
    bad_cases.append(d3)
    keep4 = {}
    d4 = _desc(m, keep4)
    keep4["vert"][keep4["ev"][0, 1]] = keep4["vert"][keep4["ev"][0, 0]] - 1.0  # inverted element
    bad_cases.append(d4)
    for d in bad_cases:
        assert L.hdg_create(ctypes.byref(d), ctypes.byref(phys), ctypes.byref(h)) == -1
    bad_phys = hdg._Phys(0.9, 0.71, 1600.0, 0.1, 5.0, 0.01, 2.0, 1)
    assert L.hdg_create(ctypes.byref(_desc(m, {})), ctypes.byref(bad_phys), ctypes.byref(h)) == -1
    assert L.hdg_create(None, ctypes.byref(phys), ctypes.byref(h)) == -1


def test_entry_points_reject_null_context():
    L = hdg.load_library()
    assert L.hdg_condense(None, 0, 1, 0, 1, None, None, None, None, 0, None) == -1
    assert L.hdg_face_matvec(None, None, None, None, None) == -1
    assert L.hdg_recover_interior(None, 0, 0, 1, None, None, None, None) == -1
    assert L.hdg_asm_block_apply(None, 0, None, None, None, None, 0, None) == -1
    assert L.hdg_local_residual_jacobian(None, 0, 1, *([None] * 8), 0, None) == -1
    assert L.hdg_bsr_pattern(None, None, None, None) == -1


def test_peak_probes_reject_bad_arguments_on_the_host():
    import ctypes
    L = hdg.load_library()
    p = ctypes.c_void_p(4096)  # never dereferenced: every call below is rejected before any launch
    q = ctypes.c_void_p(4096 + 65536)
    assert L.hdg_peak_mfma(16, 1, 1, 1.0, p, None) == -1
    assert L.hdg_peak_mfma(64, 0, 1, 1.0, p, None) == -1
    assert L.hdg_peak_mfma(32, (1 << 20) + 1, 1, 1.0, p, None) == -1
    assert L.hdg_peak_mfma(64, 1, 0, 1.0, p, None) == -1
    assert L.hdg_peak_mfma(64, 1, 1, 1.0, None, None) == -1
    assert L.hdg_peak_read(p, 0, q, None) == -1
    assert L.hdg_peak_read(p, 24, q, None) == -1
    assert L.hdg_peak_read(ctypes.c_void_p(4104), 32, q, None) == -1
    assert L.hdg_peak_read(p, 32, None, None) == -1
    assert L.hdg_peak_copy(p, q, 0, None) == -1
    assert L.hdg_peak_copy(p, q, 40, None) == -1
    assert L.hdg_peak_copy(p, ctypes.c_void_p(4096 + 1024), 2048, None) == -1  # overlapping
    assert L.hdg_peak_copy(None, q, 16, None) == -1
    assert L.hdg_status_string(-5) == b"workspace too small"
