"""Thin ctypes binding of libhdg (argument marshalling only).

Every entry point of ``include/hdg.h`` has a method of the same name on
:class:`Context`.  Arrays are torch tensors on the GPU (device memory) and the
stream is torch's current stream; all arithmetic happens in the HIP kernels of
libhdg.  There is no fallback: if the library is missing or the device is not
a GPU, construction raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdg.so")

HDG_FP64 = 0
HDG_MIXED = 1
HDG_MIXED_FAST = 2  # all-FP32 condensation, reported beside HDG_MIXED

LAYOUT = {"node_off": 0, "face_off": 1, "E_off": 2, "SK_off": 3, "bsr_row_ptr": 4, "bsr_col": 5,
          "bsr_val_off": 6, "asm_off": 7, "elem_n": 8, "elem_f": 9, "x_off": 10}

EXPORTS = ["hdg_create", "hdg_destroy", "hdg_status_string", "hdg_layout", "hdg_layout_length", "hdg_bsr_pattern",
           "hdg_workspace_size", "hdg_local_residual_jacobian", "hdg_condense", "hdg_assemble_trace",
           "hdg_face_matvec", "hdg_asm_setup", "hdg_asm_block_apply", "hdg_gmres", "hdg_recover_interior",
           "hdg_store_x", "hdg_recover_interior_x",
           "hdg_newton_step", "hdg_graph_capture_newton", "hdg_graph_launch", "hdg_graph_destroy",
           "hdg_asm_block_apply_noalloc", "hdg_gmres_x0", "hdg_rb_guess", "hdg_rb_insert", "hdg_state_update",
           "hdg_state_admissible", "hdg_lincomb", "hdg_residual_gather", "hdg_residual_norm", "hdg_av_field",
           "hdg_set_update_tile", "hdg_get_update_tile", "hdg_peak_mfma", "hdg_peak_read", "hdg_peak_copy"]

RB_MAX = 32

_vp = ctypes.c_void_p
_i = ctypes.c_int
_lib = None


class HDGError(RuntimeError):
    pass


class _MeshDesc(ctypes.Structure):
    _fields_ = [("n_elem", _i), ("n_face", _i), ("n_vert", _i), ("vert_xyz", _vp), ("elem_vert", _vp),
                ("elem_face", _vp), ("face_elem", _vp), ("face_bc", _vp), ("elem_p", _vp), ("elem_geom", _vp)]


class _Phys(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("prandtl", ctypes.c_double), ("reynolds", ctypes.c_double),
                ("mach", ctypes.c_double), ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("alpha", ctypes.c_double), ("visc_law", _i)]


class _NewtonArgs(ctypes.Structure):
    _fields_ = [("prec", _i), ("refine_steps", _i), ("asm_prec", _i), ("gmres_m", _i), ("n_chunks", _i),
                ("chunk_e0", _vp), ("chunk_ne", _vp),
                ("Q", _vp), ("U", _vp), ("Un", _vp), ("Uhat", _vp), ("nu", _vp), ("Ub", _vp),
                ("E", _vp), ("qp_work", _vp), ("qp_work_bytes", ctypes.c_size_t),
                ("cond_work", _vp), ("cond_work_bytes", ctypes.c_size_t),
                ("SK", _vp), ("info", _vp), ("S_bsr", _vp), ("g", _vp),
                ("Sinv", _vp), ("asm_info", _vp), ("asm_work", _vp), ("asm_work_bytes", ctypes.c_size_t),
                ("gmres_work", _vp), ("gmres_work_bytes", ctypes.c_size_t),
                ("dUhat", _vp), ("res_hist", _vp), ("dQU", _vp)]


class _AvParams(ctypes.Structure):
    _fields_ = [("c_av", ctypes.c_double), ("h_m", ctypes.c_double), ("eps", ctypes.c_double),
                ("s_max", ctypes.c_double), ("rho_min", ctypes.c_double), ("p_min", ctypes.c_double),
                ("smooth_iters", _i)]


def load_library(path: str = LIB_PATH):
    """Load libhdg.so (no GPU needed to load it)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HDGError(f"libhdg not built: {path} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    L.hdg_create.argtypes = [ctypes.POINTER(_MeshDesc), ctypes.POINTER(_Phys), ctypes.POINTER(_vp)]
    L.hdg_destroy.argtypes = [_vp]
    L.hdg_destroy.restype = None
    L.hdg_status_string.argtypes = [_i]
    L.hdg_status_string.restype = ctypes.c_char_p
    L.hdg_layout.argtypes = [_vp, _i, _vp, ctypes.c_int64]
    L.hdg_layout_length.argtypes = [_vp, _i]
    L.hdg_layout_length.restype = ctypes.c_int64
    L.hdg_bsr_pattern.argtypes = [_vp, ctypes.POINTER(_i), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]
    L.hdg_workspace_size.argtypes = [_vp, _i, _i, _i, _i, ctypes.POINTER(ctypes.c_size_t)]
    L.hdg_local_residual_jacobian.argtypes = [_vp, _i, _i] + [_vp] * 7 + [_vp, ctypes.c_size_t, _vp]
    L.hdg_condense.argtypes = [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.hdg_assemble_trace.argtypes = [_vp, _vp, _vp, _vp, _vp]
    L.hdg_face_matvec.argtypes = [_vp, _vp, _vp, _vp, _vp]
    L.hdg_asm_setup.argtypes = [_vp, _i, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.hdg_asm_block_apply.argtypes = [_vp, _i, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.hdg_gmres.argtypes = [_vp, _i, _vp, _vp, _vp, _i, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.hdg_recover_interior.argtypes = [_vp, _i, _i, _i, _vp, _vp, _vp, _vp]
    L.hdg_store_x.argtypes = [_vp, _i, _i, _vp, _vp, _vp]
    L.hdg_recover_interior_x.argtypes = [_vp, _i, _i, _vp, _vp, _vp, _vp]
    L.hdg_newton_step.argtypes = [_vp, ctypes.POINTER(_NewtonArgs), _vp]
    L.hdg_graph_capture_newton.argtypes = [_vp, ctypes.POINTER(_NewtonArgs), ctypes.POINTER(_vp), _vp]
    L.hdg_graph_launch.argtypes = [_vp, _vp]
    L.hdg_graph_destroy.argtypes = [_vp]
    L.hdg_graph_destroy.restype = None
    L.hdg_asm_block_apply_noalloc.argtypes = [_vp, _i, _vp, _vp, _vp, _vp]
    L.hdg_gmres_x0.argtypes = [_vp, _i, _vp, _vp, _vp, _vp, _i, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.hdg_rb_guess.argtypes = [_vp, _i, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.hdg_rb_insert.argtypes = [_vp, _vp, _vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), _vp, _vp, _vp]
    L.hdg_state_update.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, _vp]
    L.hdg_state_admissible.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp]
    L.hdg_lincomb.argtypes = [_vp, _i, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_double), _vp, ctypes.c_int64,
                              _vp]
    L.hdg_residual_gather.argtypes = [_vp, _i, _i, _vp, _vp, ctypes.c_size_t, _vp]
    L.hdg_residual_norm.argtypes = [_vp, _vp, ctypes.c_size_t, _vp, _vp]
    L.hdg_av_field.argtypes = [_vp, ctypes.POINTER(_AvParams), _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.hdg_set_update_tile.argtypes = [_vp, _i, _i]
    L.hdg_get_update_tile.argtypes = [_vp, _i]
    L.hdg_peak_mfma.argtypes = [_i, _i, _i, ctypes.c_double, _vp, _vp]
    L.hdg_peak_read.argtypes = [_vp, ctypes.c_size_t, _vp, _vp]
    L.hdg_peak_copy.argtypes = [_vp, _vp, ctypes.c_size_t, _vp]
    for name in EXPORTS:
        if name not in ("hdg_destroy", "hdg_status_string", "hdg_layout_length", "hdg_graph_destroy"):
            getattr(L, name).restype = _i
    _lib = L
    return L


def _check(rc, what):
    if rc != 0:
        msg = _lib.hdg_status_string(rc).decode()
        raise HDGError(f"{what} failed: {msg} ({rc})")


def _ptr(t, dtype=None, numel=None, name="array"):
    """Device pointer of a contiguous GPU tensor, checking dtype and size."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise HDGError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise HDGError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise HDGError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise HDGError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def hdg_peak_mfma(fp_bits, n_wg, iters, one, sink, stream=None):
    """Matrix-core peak probe (no context): n_wg * 4 * iters * 8 * 2048 flop."""
    import torch
    dt = torch.float64 if fp_bits == 64 else torch.float32
    L = load_library()
    _check(L.hdg_peak_mfma(fp_bits, n_wg, iters, float(one), _ptr(sink, dt, n_wg * 256, "sink"), _stream(stream)),
           "hdg_peak_mfma")


def hdg_peak_read(src, sink, stream=None):
    """Streaming-read probe (no context): XOR of src's 32-bit words into sink[0] (int32, zeroed by the caller)."""
    import torch
    L = load_library()
    _check(L.hdg_peak_read(_ptr(src, None, None, "src"), src.numel() * src.element_size(),
                           _ptr(sink, torch.int32, 1, "sink"), _stream(stream)), "hdg_peak_read")


def hdg_peak_copy(src, dst, stream=None):
    """Streaming-copy probe (no context): copies src into dst, 2 * bytes of traffic."""
    L = load_library()
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise HDGError("dst is smaller than src")
    _check(L.hdg_peak_copy(_ptr(src, None, None, "src"), _ptr(dst, None, None, "dst"), nbytes, _stream(stream)),
           "hdg_peak_copy")


def descriptors(mesh, wl_or_phys):
    """(hdg_mesh_desc, hdg_phys, arrays the descriptor points into) for a
    mesh and a set of physical constants (argument marshalling only)."""
    keep = dict(
        vert=np.ascontiguousarray(mesh.vert_xyz, dtype=np.float64),
        ev=np.ascontiguousarray(mesh.elem_vert, dtype=np.int32),
        ef=np.ascontiguousarray(mesh.elem_face, dtype=np.int32),
        fe=np.ascontiguousarray(mesh.face_elem, dtype=np.int32),
        bc=np.ascontiguousarray(mesh.face_bc, dtype=np.int8),
        p=np.ascontiguousarray(mesh.elem_p, dtype=np.int8))
    geom = getattr(mesh, "elem_geom", None)
    if geom is not None:
        keep["geom"] = np.ascontiguousarray(geom, dtype=np.float64).reshape(mesh.n_elem, 27, 3)
    desc = _MeshDesc(mesh.n_elem, mesh.n_face, mesh.n_vert, keep["vert"].ctypes.data, keep["ev"].ctypes.data,
                     keep["ef"].ctypes.data, keep["fe"].ctypes.data, keep["bc"].ctypes.data, keep["p"].ctypes.data,
                     keep["geom"].ctypes.data if geom is not None else None)
    w = wl_or_phys
    phys = _Phys(w.gamma, w.prandtl, w.reynolds, w.mach, w.tau, w.dt, w.alpha, int(w.visc_law))
    return desc, phys, keep


class Context:
    """An hdg_ctx for one mesh and one set of physical constants."""

    def __init__(self, mesh, wl_or_phys):
        import torch
        if not torch.cuda.is_available():
            raise HDGError("libhdg needs a GPU (torch.cuda.is_available() is False)")
        L = load_library()
        self.mesh = mesh
        desc, phys, self._keep = descriptors(mesh, wl_or_phys)
        torch.cuda.init()
        h = _vp()
        _check(L.hdg_create(ctypes.byref(desc), ctypes.byref(phys), ctypes.byref(h)), "hdg_create")
        self.h = h
        self.L = L
        self.layout = {name: self._layout(kind) for name, kind in LAYOUT.items()}
        self.n_elem = mesh.n_elem
        self.n_face = mesh.n_face
        self.N_uh = int(self.layout["face_off"][-1])

    def _layout(self, kind):
        n = self.L.hdg_layout_length(self.h, kind)
        out = np.zeros(max(n, 1), dtype=np.int64)
        _check(self.L.hdg_layout(self.h, kind, out.ctypes.data, n), "hdg_layout")
        return out[:n]

    def close(self):
        if getattr(self, "h", None):
            self.L.hdg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hdg_bsr_pattern(self):
        """(nnzb, device address of row_ptr int32[n_face+1], device address of col int32[nnzb])."""
        nnzb, rp, col = _i(), _vp(), _vp()
        _check(self.L.hdg_bsr_pattern(self.h, ctypes.byref(nnzb), ctypes.byref(rp), ctypes.byref(col)),
               "hdg_bsr_pattern")
        return nnzb.value, rp.value, col.value

    # ------------------------------------------------------------- sizes
    def workspace_size(self, op, prec=HDG_FP64, e0=0, ne=None):
        ne = self.n_elem if ne is None else ne
        out = ctypes.c_size_t()
        _check(self.L.hdg_workspace_size(self.h, op, prec, e0, ne, ctypes.byref(out)), "hdg_workspace_size")
        return out.value

    def e_size(self, e0, ne):
        if e0 < 0 or ne < 1 or e0 + ne > self.n_elem:
            return 0  # the library rejects the chunk itself
        return int(self.layout["E_off"][e0 + ne] - self.layout["E_off"][e0])

    # ------------------------------------------------------ entry points
    def hdg_local_residual_jacobian(self, e0, ne, Q, U, Un, Uhat, nu, Ub, E, work, stream=None):
        import torch
        f64 = torch.float64
        nn = int(self.layout["node_off"][-1])
        rc = self.L.hdg_local_residual_jacobian(
            self.h, e0, ne, _ptr(Q, f64, 15 * nn, "Q"), _ptr(U, f64, 5 * nn, "U"), _ptr(Un, f64, 5 * nn, "Un"),
            _ptr(Uhat, f64, self.N_uh, "Uhat"), _ptr(nu, f64, nn, "nu"),
            _ptr(Ub, f64, self.N_uh, "Ub") if Ub is not None else None,
            _ptr(E, f64, self.e_size(e0, ne), "E"), _ptr(work, None, None, "work"),
            work.numel() * work.element_size(), _stream(stream))
        _check(rc, "hdg_local_residual_jacobian")

    def hdg_condense(self, prec, refine_steps, e0, ne, E, SK, info, work, stream=None):
        import torch
        rc = self.L.hdg_condense(self.h, prec, refine_steps, e0, ne, _ptr(E, torch.float64, self.e_size(e0, ne), "E"),
                                 _ptr(SK, torch.float64, int(self.layout["SK_off"][-1]), "SK"),
                                 _ptr(info, torch.int32, self.n_elem, "info"), _ptr(work, None, None, "work"),
                                 work.numel() * work.element_size(), _stream(stream))
        _check(rc, "hdg_condense")

    def hdg_assemble_trace(self, SK, S, g, stream=None):
        import torch
        rc = self.L.hdg_assemble_trace(self.h, _ptr(SK, torch.float64, int(self.layout["SK_off"][-1]), "SK"),
                                       _ptr(S, torch.float64, int(self.layout["bsr_val_off"][-1]), "S"),
                                       _ptr(g, torch.float64, self.N_uh, "g"), _stream(stream))
        _check(rc, "hdg_assemble_trace")

    def hdg_face_matvec(self, S, x, y, stream=None):
        import torch
        rc = self.L.hdg_face_matvec(self.h, _ptr(S, torch.float64, int(self.layout["bsr_val_off"][-1]), "S"),
                                    _ptr(x, torch.float64, self.N_uh, "x"), _ptr(y, torch.float64, self.N_uh, "y"),
                                    _stream(stream))
        _check(rc, "hdg_face_matvec")

    def _sinv_dtype(self, prec):
        import torch
        return torch.float64 if prec == HDG_FP64 else torch.float32

    def hdg_asm_setup(self, prec, S, Sinv, info, work, stream=None):
        import torch
        rc = self.L.hdg_asm_setup(self.h, prec, _ptr(S, torch.float64, int(self.layout["bsr_val_off"][-1]), "S"),
                                  _ptr(Sinv, self._sinv_dtype(prec), int(self.layout["asm_off"][-1]), "Sinv"),
                                  _ptr(info, torch.int32, self.n_elem, "info"), _ptr(work, None, None, "work"),
                                  work.numel() * work.element_size(), _stream(stream))
        _check(rc, "hdg_asm_setup")

    def hdg_asm_block_apply(self, prec, Sinv, r, z, work, stream=None):
        import torch
        rc = self.L.hdg_asm_block_apply(self.h, prec,
                                        _ptr(Sinv, self._sinv_dtype(prec), int(self.layout["asm_off"][-1]), "Sinv"),
                                        _ptr(r, torch.float64, self.N_uh, "r"), _ptr(z, torch.float64, self.N_uh, "z"),
                                        _ptr(work, None, None, "work"), work.numel() * work.element_size(),
                                        _stream(stream))
        _check(rc, "hdg_asm_block_apply")

    def hdg_gmres(self, prec, S, Sinv, g, m, dUhat, res_hist, work, stream=None):
        import torch
        rc = self.L.hdg_gmres(self.h, prec, _ptr(S, torch.float64, int(self.layout["bsr_val_off"][-1]), "S"),
                              _ptr(Sinv, self._sinv_dtype(prec), int(self.layout["asm_off"][-1]), "Sinv"),
                              _ptr(g, torch.float64, self.N_uh, "g"), int(m),
                              _ptr(dUhat, torch.float64, self.N_uh, "dUhat"),
                              _ptr(res_hist, torch.float64, m + 1, "res_hist"), _ptr(work, None, None, "work"),
                              work.numel() * work.element_size(), _stream(stream))
        _check(rc, "hdg_gmres")

    def hdg_recover_interior(self, prec, e0, ne, E, dUhat, dQU, stream=None):
        import torch
        nn = int(self.layout["node_off"][-1])
        rc = self.L.hdg_recover_interior(self.h, prec, e0, ne, _ptr(E, torch.float64, self.e_size(e0, ne), "E"),
                                         _ptr(dUhat, torch.float64, self.N_uh, "dUhat"),
                                         _ptr(dQU, torch.float64, 20 * nn, "dQU"), _stream(stream))
        _check(rc, "hdg_recover_interior")

    def hdg_store_x(self, e0, ne, E, X, stream=None):
        import torch
        rc = self.L.hdg_store_x(self.h, e0, ne, _ptr(E, torch.float64, self.e_size(e0, ne), "E"),
                                _ptr(X, torch.float64, int(self.layout["x_off"][-1]), "X"), _stream(stream))
        _check(rc, "hdg_store_x")

    def hdg_recover_interior_x(self, e0, ne, X, dUhat, dQU, stream=None):
        import torch
        nn = int(self.layout["node_off"][-1])
        rc = self.L.hdg_recover_interior_x(self.h, e0, ne, _ptr(X, torch.float64, int(self.layout["x_off"][-1]), "X"),
                                           _ptr(dUhat, torch.float64, self.N_uh, "dUhat"),
                                           _ptr(dQU, torch.float64, 20 * nn, "dQU"), _stream(stream))
        _check(rc, "hdg_recover_interior_x")

    def hdg_asm_block_apply_noalloc(self, prec, Sinv, r, z, stream=None):
        import torch
        rc = self.L.hdg_asm_block_apply_noalloc(
            self.h, prec, _ptr(Sinv, self._sinv_dtype(prec), int(self.layout["asm_off"][-1]), "Sinv"),
            _ptr(r, torch.float64, self.N_uh, "r"), _ptr(z, torch.float64, self.N_uh, "z"), _stream(stream))
        _check(rc, "hdg_asm_block_apply_noalloc")

    # ------------------------------------------------- solver-loop calls
    def hdg_gmres_x0(self, prec, S, Sinv, g, x0, m, dUhat, res_hist, work, stream=None):
        import torch
        f64 = torch.float64
        rc = self.L.hdg_gmres_x0(self.h, prec, _ptr(S, f64, int(self.layout["bsr_val_off"][-1]), "S"),
                                 _ptr(Sinv, self._sinv_dtype(prec), int(self.layout["asm_off"][-1]), "Sinv"),
                                 _ptr(g, f64, self.N_uh, "g"), _ptr(x0, f64, self.N_uh, "x0"), int(m),
                                 _ptr(dUhat, f64, self.N_uh, "dUhat"), _ptr(res_hist, f64, m + 1, "res_hist"),
                                 _ptr(work, None, None, "work"), work.numel() * work.element_size(), _stream(stream))
        _check(rc, "hdg_gmres_x0")

    def hdg_rb_guess(self, nb, W, Z, g, x0, work, stream=None):
        import torch
        f64 = torch.float64
        rc = self.L.hdg_rb_guess(self.h, int(nb), _ptr(W, f64, nb * self.N_uh, "W") if nb else None,
                                 _ptr(Z, f64, nb * self.N_uh, "Z") if nb else None, _ptr(g, f64, self.N_uh, "g"),
                                 _ptr(x0, f64, self.N_uh, "x0"), _ptr(work, None, None, "work") if work is not None
                                 else None, 0 if work is None else work.numel() * work.element_size(),
                                 _stream(stream))
        _check(rc, "hdg_rb_guess")

    def hdg_rb_insert(self, S, w_new, nb_max, count, head, W, Z, stream=None):
        """Returns the new (count, head)."""
        import torch
        f64 = torch.float64
        c, h = _i(count), _i(head)
        rc = self.L.hdg_rb_insert(self.h, _ptr(S, f64, int(self.layout["bsr_val_off"][-1]), "S"),
                                  _ptr(w_new, f64, self.N_uh, "w_new"), int(nb_max), ctypes.byref(c), ctypes.byref(h),
                                  _ptr(W, f64, nb_max * self.N_uh, "W"), _ptr(Z, f64, nb_max * self.N_uh, "Z"),
                                  _stream(stream))
        _check(rc, "hdg_rb_insert")
        return c.value, h.value

    def hdg_state_update(self, alpha, dQU, dUhat, Q, U, Uhat, stream=None):
        import torch
        f64 = torch.float64
        nn = int(self.layout["node_off"][-1])
        rc = self.L.hdg_state_update(self.h, float(alpha), _ptr(dQU, f64, 20 * nn, "dQU"),
                                     _ptr(dUhat, f64, self.N_uh, "dUhat"), _ptr(Q, f64, 15 * nn, "Q"),
                                     _ptr(U, f64, 5 * nn, "U"), _ptr(Uhat, f64, self.N_uh, "Uhat"), _stream(stream))
        _check(rc, "hdg_state_update")

    def hdg_state_admissible(self, alpha, U, dQU, flag, stream=None):
        import torch
        nn = int(self.layout["node_off"][-1])
        rc = self.L.hdg_state_admissible(self.h, float(alpha), _ptr(U, torch.float64, 5 * nn, "U"),
                                         _ptr(dQU, torch.float64, 20 * nn, "dQU"), _ptr(flag, torch.int32, 1, "flag"),
                                         _stream(stream))
        _check(rc, "hdg_state_admissible")

    def hdg_lincomb(self, vecs, coefs, out, stream=None):
        import torch
        n = out.numel()
        vs = (_vp * len(vecs))(*[_ptr(v, torch.float64, n, "v") for v in vecs])
        cs = (ctypes.c_double * len(coefs))(*[float(c) for c in coefs])
        rc = self.L.hdg_lincomb(self.h, len(vecs), vs, cs, _ptr(out, torch.float64, n, "out"), n, _stream(stream))
        _check(rc, "hdg_lincomb")

    def hdg_residual_gather(self, e0, ne, E, work, stream=None):
        import torch
        rc = self.L.hdg_residual_gather(self.h, e0, ne, _ptr(E, torch.float64, self.e_size(e0, ne), "E"),
                                        _ptr(work, None, None, "work"), work.numel() * work.element_size(),
                                        _stream(stream))
        _check(rc, "hdg_residual_gather")

    def hdg_residual_norm(self, work, norms, stream=None):
        import torch
        rc = self.L.hdg_residual_norm(self.h, _ptr(work, None, None, "work"), work.numel() * work.element_size(),
                                      _ptr(norms, torch.float64, 3, "norms"), _stream(stream))
        _check(rc, "hdg_residual_norm")

    def hdg_av_field(self, params, U, Q, nu, work, nu_raw=None, stream=None):
        """params: dict with c_av, h_m, eps, s_max, rho_min, p_min, smooth_iters."""
        import torch
        f64 = torch.float64
        nn = int(self.layout["node_off"][-1])
        ap = _AvParams(float(params["c_av"]), float(params["h_m"]), float(params["eps"]), float(params["s_max"]),
                       float(params["rho_min"]), float(params["p_min"]), int(params["smooth_iters"]))
        rc = self.L.hdg_av_field(self.h, ctypes.byref(ap), _ptr(U, f64, 5 * nn, "U"), _ptr(Q, f64, 15 * nn, "Q"),
                                 _ptr(nu_raw, f64, self.n_elem, "nu_raw") if nu_raw is not None else None,
                                 _ptr(nu, f64, nn, "nu"), _ptr(work, None, None, "work"),
                                 work.numel() * work.element_size(), _stream(stream))
        _check(rc, "hdg_av_field")

    def hdg_set_update_tile(self, n, tile_rows):
        _check(self.L.hdg_set_update_tile(self.h, int(n), int(tile_rows)), "hdg_set_update_tile")

    def hdg_get_update_tile(self, n):
        rc = self.L.hdg_get_update_tile(self.h, int(n))
        if rc < 0:
            _check(rc, "hdg_get_update_tile")
        return rc

    # ------------------------------------------------------- whole step
    def newton_args(self, st):
        """hdg_newton_args for a pipeline.NewtonStep's buffers (the struct and
        the host chunk arrays are kept alive on the returned object)."""
        import torch
        f64 = torch.float64
        nn = int(self.layout["node_off"][-1])
        e0 = np.ascontiguousarray([c[0] for c in st.chunks], dtype=np.int32)
        ne = np.ascontiguousarray([c[1] for c in st.chunks], dtype=np.int32)
        nb = lambda t: t.numel() * t.element_size()
        a = _NewtonArgs(
            st.prec, st.refine, st.asm_prec, st.m, len(st.chunks), e0.ctypes.data, ne.ctypes.data,
            _ptr(st.Q, f64, 15 * nn, "Q"), _ptr(st.U, f64, 5 * nn, "U"), _ptr(st.Un, f64, 5 * nn, "Un"),
            _ptr(st.Uhat, f64, self.N_uh, "Uhat"), _ptr(st.nu, f64, nn, "nu"),
            _ptr(st.Ub, f64, self.N_uh, "Ub") if st.Ub is not None else None,
            _ptr(st.E, f64, int(self.layout["E_off"][-1]), "E"), _ptr(st.qp_work), nb(st.qp_work),
            _ptr(st.cond_work), nb(st.cond_work),
            _ptr(st.SK, f64, int(self.layout["SK_off"][-1]), "SK"), _ptr(st.info, torch.int32, self.n_elem, "info"),
            _ptr(st.S, f64, int(self.layout["bsr_val_off"][-1]), "S"), _ptr(st.g, f64, self.N_uh, "g"),
            _ptr(st.Sinv, self._sinv_dtype(st.asm_prec), int(self.layout["asm_off"][-1]), "Sinv"),
            _ptr(st.asm_info, torch.int32, self.n_elem, "asm_info"), _ptr(st.asm_work), nb(st.asm_work),
            _ptr(st.gm_work), nb(st.gm_work),
            _ptr(st.dUhat, f64, self.N_uh, "dUhat"), _ptr(st.hist, f64, st.m + 1, "res_hist"),
            _ptr(st.dQU, f64, 20 * nn, "dQU"))
        a._keep = (e0, ne)
        return a

    def hdg_newton_step(self, args, stream=None):
        _check(self.L.hdg_newton_step(self.h, ctypes.byref(args), _stream(stream)), "hdg_newton_step")

    def hdg_graph_capture_newton(self, args, stream):
        """Capture the whole step on `stream` (a created torch.cuda.Stream, not
        the default stream); returns a Graph."""
        g = _vp()
        _check(self.L.hdg_graph_capture_newton(self.h, ctypes.byref(args), ctypes.byref(g), _stream(stream)),
               "hdg_graph_capture_newton")
        return Graph(self, g, args)


class Graph:
    """A captured Newton step (hdg_graph); replay() enqueues one launch."""

    def __init__(self, ctx, handle, args):
        self.ctx = ctx
        self.h = handle
        self._args = args  # the captured pointers belong to these buffers

    def replay(self, stream=None):
        _check(self.ctx.L.hdg_graph_launch(self.h, _stream(stream)), "hdg_graph_launch")

    def close(self):
        if getattr(self, "h", None):
            self.ctx.L.hdg_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
