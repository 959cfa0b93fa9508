"""CPU oracle of the HDG element-local hot path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP path:
the element systems and the condensation come from ``hdgref.c`` (plain C,
dual-number Jacobians, textbook LU), the trace-space algebra below is written
out with numpy from the paper's definitions:

* assembly of the condensed trace system S dUhat = g (eq. schur-trace) from the
  element Schur complements S^K = D - C A^{-1} B and g^K = -R_uh + C A^{-1} R_qu
  (eqs. newton-local-block, local-elimination);
* the one-level additive Schwarz preconditioner with element-centred face
  patches, M^{-1} = sum_r R_r^T S_r^{-1} R_r (eq. additive-schwarz);
* restarted, left-preconditioned GMRES with modified Gram-Schmidt and Givens
  rotations (section "Parallel Newton-GMRES Solver");
* recovery of the interior correction (eq. local-elimination).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hdgref.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile hdgref.c with gcc (host only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            L.hdgref_element_system.argtypes = [ctypes.c_int, _ip, _ip, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                                _dp, _dp, _dp, _dp]
            L.hdgref_element_system.restype = ctypes.c_int
            L.hdgref_condense.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp]
            L.hdgref_condense.restype = ctypes.c_int
            L.hdgref_dense_solve.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int]
            L.hdgref_dense_solve.restype = ctypes.c_int
            L.hdgref_lu_factor.argtypes = [ctypes.c_int, _dp, _ip]
            L.hdgref_lu_factor.restype = ctypes.c_int
            L.hdgref_lu_solve.argtypes = [ctypes.c_int, _dp, _ip, _dp, ctypes.c_int]
            L.hdgref_lu_solve.restype = None
            L.hdgref_gauss.argtypes = [ctypes.c_int, _dp, _dp]
            L.hdgref_gll.argtypes = [ctypes.c_int, _dp]
            L.hdgref_point_flux.argtypes = [_dp, _dp, ctypes.c_double, _dp, _dp, _dp, _dp, _dp]
            L.hdgref_element_volume.argtypes = [ctypes.c_int, ctypes.c_int, _dp]
            L.hdgref_element_volume.restype = ctypes.c_double
            _lib = L
    return _lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------ 1-D rules
def gauss(nq):
    x, w = np.zeros(nq), np.zeros(nq)
    lib().hdgref_gauss(nq, _p(x), _p(w))
    return x, w


def gll(p):
    x = np.zeros(p + 1)
    lib().hdgref_gll(p, _p(x))
    return x


def params(wl):
    return np.array([wl.gamma, wl.prandtl, wl.reynolds, wl.mach, wl.tau, wl.dt, wl.alpha,
                     float(wl.visc_law)])


def point_flux(w5, q15, nu, prm):
    """Fc, Fv [5,3] and their derivatives [5,3,20] w.r.t. (u 0..4, q 5..19)."""
    Fc, Fv = np.zeros(15), np.zeros(15)
    dFc, dFv = np.zeros(300), np.zeros(300)
    lib().hdgref_point_flux(_p(_f64(w5)), _p(_f64(q15)), float(nu), _p(_f64(prm)),
                            _p(Fc), _p(Fv), _p(dFc), _p(dFv))
    return Fc.reshape(5, 3), Fv.reshape(5, 3), dFc.reshape(5, 3, 20), dFv.reshape(5, 3, 20)


# ------------------------------------------------------- element systems
class Sizes:
    """Per-element sizes and offsets of a workload's mesh."""

    def __init__(self, mesh):
        self.mesh = mesh
        self.fp = mesh.face_p()
        self.noff = mesh.node_offsets()
        self.foff = mesh.face_offsets()

    def Np(self, e):
        return (int(self.mesh.elem_p[e]) + 1) ** 3

    def face_sizes(self, e):
        return [5 * (int(self.fp[F]) + 1) ** 2 for F in self.mesh.elem_face[e]]

    def n(self, e):
        return 20 * self.Np(e)

    def f(self, e):
        return sum(self.face_sizes(e))


def gather_trace(wl, sizes, e, vec):
    """Element-local trace vector [sum_lf 5 N_fp] from a global face vector."""
    out = []
    for F in wl.mesh.elem_face[e]:
        out.append(vec[sizes.foff[F]:sizes.foff[F + 1]])
    return np.concatenate(out)


def element_geometry(mesh, e):
    """(order, nodes) of element e's geometry map: the 8 vertices (trilinear), or
    the mesh's 27 curved-geometry nodes (triquadratic) when it has them."""
    geom = getattr(mesh, "elem_geom", None)
    if geom is None:
        return 1, _f64(mesh.vert_xyz[mesh.elem_vert[e]].ravel())
    return 2, _f64(np.asarray(geom[e]).ravel())


def element_volume(mesh, e):
    g, Xg = element_geometry(mesh, e)
    return lib().hdgref_element_volume(int(mesh.elem_p[e]), g, _p(Xg))


def element_system(wl, e, sizes=None, U=None, Q=None, Uhat=None):
    """E^K = [[A, B, R_qu], [C, D, R_uh]] of element e (column-major, (n+f) x (n+f+1))."""
    sizes = sizes or Sizes(wl.mesh)
    m = wl.mesh
    U = wl.U if U is None else U
    Q = wl.Q if Q is None else Q
    Uhat = wl.Uhat if Uhat is None else Uhat
    p = int(m.elem_p[e])
    Np = (p + 1) ** 3
    o = sizes.noff[e]
    pf = np.array([sizes.fp[F] for F in m.elem_face[e]], dtype=np.int32)
    bc = np.array([m.face_bc[F] for F in m.elem_face[e]], dtype=np.int32)
    g, Xg = element_geometry(m, e)
    n = 20 * Np
    f = sizes.f(e)
    E = np.zeros((n + f + 1) * (n + f))
    rc = lib().hdgref_element_system(
        p, _p(pf, _ip), _p(bc, _ip), g, _p(Xg), _p(params(wl)),
        _p(_f64(Q[15 * o:15 * (o + Np)])), _p(_f64(U[5 * o:5 * (o + Np)])),
        _p(_f64(wl.Un[5 * o:5 * (o + Np)])), _p(_f64(wl.nu[o:o + Np])),
        _p(_f64(gather_trace(wl, sizes, e, Uhat))), _p(_f64(gather_trace(wl, sizes, e, wl.Ub))),
        _p(E))
    assert rc == 0
    return E.reshape(n + f + 1, n + f).T  # view: E[row, col]


def split(E, n):
    """A, B, C, D, R_qu, R_uh views of an element system."""
    f = E.shape[0] - n
    return E[:n, :n], E[:n, n:n + f], E[n:, :n], E[n:, n:n + f], E[:n, n + f], E[n:, n + f]


def condense(E, n):
    """(S^K [f,f], g^K [f], X [n, f+1]) by the oracle's LU."""
    f = E.shape[0] - n
    buf = np.ascontiguousarray(E.T)  # column-major storage of E
    SK = np.zeros(f * f)
    gK = np.zeros(f)
    X = np.zeros(n * (f + 1))
    info = lib().hdgref_condense(n, f, _p(buf), _p(SK), _p(gK), _p(X))
    assert info == 0, info
    return SK.reshape(f, f).T.copy(), gK, X.reshape(f + 1, n).T.copy()


def dense_solve(A, b):
    """Oracle LU solve (own code) of A x = b; b may be 1-D or 2-D."""
    A = np.asfortranarray(A, dtype=np.float64).copy(order="F")
    bb = np.asfortranarray(b.reshape(b.shape[0], -1), dtype=np.float64).copy(order="F")
    info = lib().hdgref_dense_solve(A.shape[0], A.ctypes.data_as(_dp), bb.ctypes.data_as(_dp),
                                    bb.shape[1])
    assert info == 0, info
    return bb.reshape(b.shape)


class LU:
    """LU factors with partial pivoting (the oracle's own code) of a dense
    matrix, kept for repeated solves."""

    def __init__(self, A):
        self.n = A.shape[0]
        self.a = np.asfortranarray(A, dtype=np.float64).copy(order="F")
        self.piv = np.zeros(self.n, dtype=np.int32)
        info = lib().hdgref_lu_factor(self.n, self.a.ctypes.data_as(_dp), self.piv.ctypes.data_as(_ip))
        assert info == 0, info

    def solve(self, b):
        bb = np.asfortranarray(b.reshape(b.shape[0], -1), dtype=np.float64).copy(order="F")
        lib().hdgref_lu_solve(self.n, self.a.ctypes.data_as(_dp), self.piv.ctypes.data_as(_ip),
                              bb.ctypes.data_as(_dp), bb.shape[1])
        return bb.reshape(b.shape)


def element_systems(wl, elems=None, threads=None):
    sizes = Sizes(wl.mesh)
    elems = range(wl.mesh.n_elem) if elems is None else elems
    with ThreadPoolExecutor(max_workers=threads or os.cpu_count()) as ex:
        return list(ex.map(lambda e: element_system(wl, e, sizes), elems))


# ------------------------------------------------------ condensed system
class TraceSystem:
    """Assembled S (blocks keyed by (F, F')) and g, from per-element S^K, g^K."""

    def __init__(self, wl, SKs, gKs):
        self.wl = wl
        self.sizes = sizes = Sizes(wl.mesh)
        m = wl.mesh
        self.N = int(sizes.foff[-1])
        self.blocks = {}
        self.g = np.zeros(self.N)
        for e in range(m.n_elem):
            fs = sizes.face_sizes(e)
            t = np.concatenate([[0], np.cumsum(fs)])
            for a, Fa in enumerate(m.elem_face[e]):
                self.g[sizes.foff[Fa]:sizes.foff[Fa + 1]] += gKs[e][t[a]:t[a + 1]]
                for b, Fb in enumerate(m.elem_face[e]):
                    blk = SKs[e][t[a]:t[a + 1], t[b]:t[b + 1]]
                    key = (int(Fa), int(Fb))
                    if key in self.blocks:
                        self.blocks[key] = self.blocks[key] + blk
                    else:
                        self.blocks[key] = blk.copy()
        self.asm_inv = None

    @classmethod
    def from_blocks(cls, wl, blocks, g):
        """A trace system with given blocks {(F, G): array} and right-hand side g."""
        ts = cls.__new__(cls)
        ts.wl = wl
        ts.sizes = Sizes(wl.mesh)
        ts.N = int(ts.sizes.foff[-1])
        ts.blocks = {k: np.array(v, dtype=np.float64) for k, v in blocks.items()}
        ts.g = np.array(g, dtype=np.float64)
        ts.asm_inv = None
        return ts

    def matvec(self, x):
        y = np.zeros(self.N)
        fo = self.sizes.foff
        for (Fa, Fb), blk in self.blocks.items():
            y[fo[Fa]:fo[Fa + 1]] += blk @ x[fo[Fb]:fo[Fb + 1]]
        return y

    def dense(self):
        S = np.zeros((self.N, self.N))
        fo = self.sizes.foff
        for (Fa, Fb), blk in self.blocks.items():
            S[fo[Fa]:fo[Fa + 1], fo[Fb]:fo[Fb + 1]] += blk
        return S

    def patch_index(self, r):
        fo = self.sizes.foff
        return np.concatenate([np.arange(fo[F], fo[F + 1]) for F in self.wl.mesh.elem_face[r]])

    def patch_matrix(self, r):
        """S_r = R_r S R_r^T on element r's six faces."""
        faces = self.wl.mesh.elem_face[r]
        rows = []
        for Fa in faces:
            rows.append(np.concatenate([self.blocks[(int(Fa), int(Fb))] for Fb in faces], axis=1))
        return np.concatenate(rows, axis=0)

    def asm_factor(self, threads=None):
        """LU factors of every S_r (kept: GMRES applies M^{-1} once per iteration)."""
        if self.asm_inv is None:
            nthr = threads or min(16, os.cpu_count() or 1)
            with ThreadPoolExecutor(max_workers=nthr) as ex:
                self.asm_inv = list(ex.map(lambda r: LU(self.patch_matrix(r)), range(self.wl.mesh.n_elem)))
        return self.asm_inv

    def asm_apply(self, y):
        """z = sum_r R_r^T S_r^{-1} R_r y (plain additive, no coarse space)."""
        z = np.zeros(self.N)
        fac = self.asm_factor()
        for r in range(self.wl.mesh.n_elem):
            idx = self.patch_index(r)
            np.add.at(z, idx, fac[r].solve(y[idx]))
        return z


def gmres(ts: TraceSystem, g, m, tol=0.0, x0=None, restarts=1):
    """Restarted, left-preconditioned GMRES(m) (section 3.2): each cycle
    minimises ||M^{-1}(g - S x)||_2 over x0 + K_m(M^{-1}S, M^{-1}(g - S x0)) by
    modified Gram-Schmidt Arnoldi, Givens rotations and back substitution; up
    to `restarts` cycles, stopping once the preconditioned residual is at most
    tol times the initial one.  x0 = 0 unless given.  Returns (x, history of
    ||M^{-1}(g - S x_j)|| over all iterations)."""
    N = g.shape[0]
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    hist = []
    beta0 = None
    for cycle in range(restarts):
        r0 = ts.asm_apply(g - ts.matvec(x)) if (x0 is not None or cycle > 0) else ts.asm_apply(g)
        beta = np.linalg.norm(r0)
        if beta0 is None:
            beta0 = beta
            hist.append(beta)
        if beta == 0.0 or (tol > 0.0 and cycle > 0 and beta <= tol * beta0):
            break
        V = np.zeros((m + 1, N))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        gam = np.zeros(m + 1)
        gam[0] = beta
        V[0] = r0 / beta
        k = 0
        for j in range(m):
            w = ts.asm_apply(ts.matvec(V[j]))
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gam[j + 1] = -sn[j] * gam[j]
            gam[j] = cs[j] * gam[j]
            hist.append(abs(gam[j + 1]))
            k = j + 1
            if tol > 0.0 and abs(gam[j + 1]) <= tol * beta0:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (gam[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + V[:k].T @ y
        if tol > 0.0 and hist[-1] <= tol * beta0:
            break
    return x, np.array(hist)


def recover(wl, sizes, e, X, dUhat):
    """d(Q,U)^K = -(x_r + X_B dUhat^K)."""
    d = gather_trace(wl, sizes, e, dUhat)
    f = d.shape[0]
    return -(X[:, f] + X[:, :f] @ d)
