"""Seeded synthetic inputs: hexahedral meshes, flow states, artificial-viscosity
fields and trace vectors.

This module is the only code shared between the HIP path and the CPU oracle.
It holds none of the HDG method's arithmetic: it places analytic fields at
node positions and draws seeded random numbers.  Node positions use the
Gauss-Lobatto points of the tensor basis (library roots of P'_p) and the
trilinear vertex map, only so that the nodal values sample a smooth field.

Workloads (nondimensional; rho_0 = 1, |v_0| = 1, L = 1, T_0 = 1):

* supersonic / subsonic Taylor-Green vortex on the periodic cube (0, 2 pi)^3
  (paper section 5.1, initial velocity, temperature and pressure equations);
* a wall-normal stretched, perturbed box with a boundary-layer-like profile
  for the mixed-degree batching case.

Each state consists of the nodal conserved variables U = (rho, rho v, rho E),
the previous-step state Un, the gradient Q = grad u (analytic, by complex
step), the face trace Uhat, and the frozen artificial viscosity nu.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

GAMMA = 1.4
PRANDTL = 0.71
TAU = 5.0
DT = 1.0e-2
# Stage 1 of Alexander's three-stage L-stable DIRK: a11 is the root in (0, 1)
# of x^3 - 3x^2 + 1.5x - 1/6; the stage mass coefficient is d11 = 1 / a11.
_A11 = 0.43586652150845899941601945


def dirk_alpha() -> float:
    return 1.0 / _A11


def gll_points(p: int) -> np.ndarray:
    """Gauss-Lobatto points on [-1, 1]: -1, roots of P_p', +1 (numpy roots)."""
    if p == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


@dataclasses.dataclass
class Mesh:
    """Conforming hex mesh, all elements identically oriented.

    elem_vert[e] lists 8 vertices in tensor order (x fastest); elem_face[e]
    the global faces on local sides -x,+x,-y,+y,-z,+z; face_elem[F] =
    [[elem, local face] of side 0, [elem, local face] of side 1], side 1 is
    [-1, -1] on a boundary face.  Side 0 is the element the face normal points
    out of.  face_bc is 0 for interior/periodic faces, else the boundary type
    (1 prescribed state, 2 extrapolated, 3 isothermal wall, 4 adiabatic wall,
    5 symmetry; box_mesh marks every non-periodic side 1).
    """

    vert_xyz: np.ndarray   # [n_vert, 3] float64
    elem_vert: np.ndarray  # [n_elem, 8] int32
    elem_face: np.ndarray  # [n_elem, 6] int32
    face_elem: np.ndarray  # [n_face, 2, 2] int32
    face_bc: np.ndarray    # [n_face] int8
    elem_p: np.ndarray     # [n_elem] int8
    shape: tuple
    elem_geom: Optional[np.ndarray] = None  # [n_elem, 27, 3] curved geometry nodes, or None (trilinear)

    @property
    def n_elem(self) -> int:
        return int(self.elem_vert.shape[0])

    @property
    def n_face(self) -> int:
        return int(self.face_elem.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.vert_xyz.shape[0])

    def face_p(self) -> np.ndarray:
        """Face degree = max of the degrees of its sides."""
        p = np.zeros(self.n_face, dtype=np.int32)
        for s in range(2):
            e = self.face_elem[:, s, 0]
            ok = e >= 0
            p[ok] = np.maximum(p[ok], self.elem_p[e[ok]])
        return p

    # --- packed-array offsets (elements / faces of differing degree) ---
    def node_offsets(self) -> np.ndarray:
        npn = (self.elem_p.astype(np.int64) + 1) ** 3
        return np.concatenate([[0], np.cumsum(npn)])

    def face_offsets(self) -> np.ndarray:
        nf = 5 * (self.face_p().astype(np.int64) + 1) ** 2
        return np.concatenate([[0], np.cumsum(nf)])


def box_mesh(n: tuple, lengths=(2 * math.pi,) * 3, periodic=(True, True, True),
             y_coords: Optional[np.ndarray] = None, perturb: float = 0.0,
             p=2, seed: int = 0) -> Mesh:
    """Structured nx*ny*nz hex mesh of a box.

    ``perturb`` displaces every vertex not on a non-periodic wall by
    U(-1, 1) * perturb * (local spacing) per axis; displacements are periodic
    so that paired periodic faces stay translates of each other.  ``p`` is an
    int or an array of per-element degrees.
    """
    nx, ny, nz = n
    xs = [np.linspace(0.0, lengths[0], nx + 1),
          np.linspace(0.0, lengths[1], ny + 1) if y_coords is None else np.asarray(y_coords, float),
          np.linspace(0.0, lengths[2], nz + 1)]
    assert len(xs[1]) == ny + 1
    I, J, K = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    vid = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
    nv = (nx + 1) * (ny + 1) * (nz + 1)
    vert = np.zeros((nv, 3))
    ii, jj, kk = I.ravel(), J.ravel(), K.ravel()
    ids = vid(ii, jj, kk)
    vert[ids, 0] = xs[0][ii]
    vert[ids, 1] = xs[1][jj]
    vert[ids, 2] = xs[2][kk]
    if perturb > 0.0:
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
        if periodic[0] and periodic[2]:
            disp = rng.uniform(-1.0, 1.0, size=(nx, ny + 1, nz, 3))
            if periodic[1]:
                disp = disp[:, :ny, :, :]
        else:  # walls across x or z too: one draw per vertex of the box
            disp = rng.uniform(-1.0, 1.0, size=(nx + 1, ny + 1, nz + 1, 3))
        dims3 = (nx, ny, nz)
        for v in range(nv):
            i, j, k = ii[v], jj[v], kk[v]
            if any(not periodic[a] and idx in (0, dims3[a]) for a, idx in enumerate((i, j, k))):
                continue
            di = disp[tuple(idx % dims3[a] if periodic[a] else idx for a, idx in enumerate((i, j, k)))]
            hloc = np.empty(3)
            for a, (idx, nn) in enumerate(((i, nx), (j, ny), (k, nz))):
                if periodic[a]:
                    c = idx % nn
                    hloc[a] = xs[a][c + 1] - xs[a][c]
                else:
                    hloc[a] = min(xs[a][idx + 1] - xs[a][idx], xs[a][idx] - xs[a][idx - 1])
            vert[v] += perturb * di * hloc
    ne = nx * ny * nz
    eid = lambda i, j, k: i + nx * (j + ny * k)
    ev = np.zeros((ne, 8), dtype=np.int32)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                e = eid(i, j, k)
                c = 0
                for dk in (0, 1):
                    for dj in (0, 1):
                        for di in (0, 1):
                            ev[e, c] = vid(i + di, j + dj, k + dk)
                            c += 1
    # faces, grouped by direction
    faces = []
    ef = -np.ones((ne, 6), dtype=np.int32)
    bc = []
    dims = (nx, ny, nz)
    for d in range(3):
        nd = dims[d]
        layers = nd if periodic[d] else nd + 1
        rng_shape = list(dims)
        rng_shape[d] = layers
        for k in range(rng_shape[2]):
            for j in range(rng_shape[1]):
                for i in range(rng_shape[0]):
                    idx = [i, j, k]
                    L = idx[d]
                    plus = list(idx)
                    minus = list(idx)
                    minus[d] = L - 1
                    if periodic[d]:
                        minus[d] %= nd
                        e_minus, e_plus = eid(*minus), eid(*plus)
                        sides = [[e_minus, 2 * d + 1], [e_plus, 2 * d]]
                        b = 0
                    else:
                        if L == 0:
                            sides = [[eid(*plus), 2 * d], [-1, -1]]
                            b = 1
                        elif L == nd:
                            sides = [[eid(*minus), 2 * d + 1], [-1, -1]]
                            b = 1
                        else:
                            sides = [[eid(*minus), 2 * d + 1], [eid(*plus), 2 * d]]
                            b = 0
                    F = len(faces)
                    faces.append(sides)
                    bc.append(b)
                    for s in sides:
                        if s[0] >= 0:
                            ef[s[0], s[1]] = F
    face_elem = np.array(faces, dtype=np.int32)
    assert (ef >= 0).all()
    if np.isscalar(p):
        ep = np.full(ne, int(p), dtype=np.int8)
    else:
        ep = np.asarray(p, dtype=np.int8)
        assert ep.shape == (ne,)
    return Mesh(vert, ev, ef, face_elem, np.array(bc, dtype=np.int8), ep, (nx, ny, nz))


# ---------------------------------------------------------------- positions
def group_by_degree(mesh: Mesh) -> Mesh:
    """The same mesh with its elements renumbered by degree (stable): every
    degree is one contiguous range of elements, so that a batch of one degree
    (one size of element system) can be condensed by launches of its own."""
    perm = np.argsort(mesh.elem_p, kind="stable")
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    fe = mesh.face_elem.copy()
    for side in range(2):
        e = fe[:, side, 0]
        ok = e >= 0
        e[ok] = inv[e[ok]]
        fe[:, side, 0] = e
    geom = None if mesh.elem_geom is None else np.ascontiguousarray(mesh.elem_geom[perm])
    return dataclasses.replace(mesh, elem_geom=geom, elem_vert=np.ascontiguousarray(mesh.elem_vert[perm]),
                               elem_face=np.ascontiguousarray(mesh.elem_face[perm]),
                               face_elem=fe, elem_p=np.ascontiguousarray(mesh.elem_p[perm]))


def set_boundary_types(mesh: Mesh, types: dict) -> Mesh:
    """The same mesh with the boundary type of each one-sided face chosen by the
    side of the box it lies on: types[(axis, side)] for axis 0..2 and side 0
    (low) or 1 (high); unlisted sides keep their type."""
    bc = mesh.face_bc.copy()
    for F in range(mesh.n_face):
        if mesh.face_elem[F, 1, 0] >= 0:
            continue
        lf = int(mesh.face_elem[F, 0, 1])
        key = (lf // 2, lf % 2)
        if key in types:
            bc[F] = types[key]
    return dataclasses.replace(mesh, face_bc=bc)


def _trilinear(X8: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Map reference points xi [..., 3] in [-1,1]^3 with vertex coords X8 [8, 3]."""
    out = np.zeros(xi.shape[:-1] + (3,))
    for v in range(8):
        b = [(v >> d) & 1 for d in range(3)]
        w = np.ones(xi.shape[:-1])
        for d in range(3):
            w = w * (0.5 * (1 + xi[..., d]) if b[d] else 0.5 * (1 - xi[..., d]))
        out += w[..., None] * X8[v]
    return out


def _triquadratic(X27: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Map reference points xi [..., 3] through 27 nodes (tensor order, at
    reference coordinates -1, 0, 1)."""
    def lq(t):
        return [0.5 * t * (t - 1.0), 1.0 - t * t, 0.5 * t * (t + 1.0)]
    L = [lq(xi[..., d]) for d in range(3)]
    out = np.zeros(xi.shape[:-1] + (3,))
    for c in range(3):
        for b in range(3):
            for a in range(3):
                out += (L[0][a] * L[1][b] * L[2][c])[..., None] * X27[a + 3 * (b + 3 * c)]
    return out


def _map(mesh: Mesh, e: int, xi: np.ndarray) -> np.ndarray:
    if mesh.elem_geom is not None:
        return _triquadratic(np.asarray(mesh.elem_geom[e]), xi)
    return _trilinear(mesh.vert_xyz[mesh.elem_vert[e]], xi)


def curve_mesh(mesh: Mesh, amp: float) -> Mesh:
    """The same mesh with curved (triquadratic) elements: the 27 nodes of each
    element are its straight (trilinear) node positions moved by the smooth
    displacement amp * (sin y sin z, sin z sin x, sin x sin y), which is
    2 pi-periodic, so shared and periodic faces stay conforming."""
    r = np.array([-1.0, 0.0, 1.0])
    Z, Y, X = np.meshgrid(r, r, r, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    geom = np.zeros((mesh.n_elem, 27, 3))
    for e in range(mesh.n_elem):
        x = _trilinear(mesh.vert_xyz[mesh.elem_vert[e]], xi)
        d = np.stack([np.sin(x[:, 1]) * np.sin(x[:, 2]), np.sin(x[:, 2]) * np.sin(x[:, 0]),
                      np.sin(x[:, 0]) * np.sin(x[:, 1])], axis=-1)
        geom[e] = x + amp * d
    return dataclasses.replace(mesh, elem_geom=geom)


def element_node_xyz(mesh: Mesh, e: int) -> np.ndarray:
    """[N_p, 3] node positions of element e, tensor order x fastest."""
    p = int(mesh.elem_p[e])
    r = gll_points(p)
    Z, Y, X = np.meshgrid(r, r, r, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=-1)
    return _map(mesh, e, xi)


def face_node_xyz(mesh: Mesh, F: int) -> np.ndarray:
    """[N_fp, 3] trace-node positions of face F (degree = max of its sides),
    seen from side 0; tangential axes in increasing direction order."""
    pf = int(mesh.face_p()[F])
    e, lf = mesh.face_elem[F, 0]
    d, s = lf // 2, lf % 2
    t = [a for a in range(3) if a != d]
    r = gll_points(pf)
    A1, A0 = np.meshgrid(r, r, indexing="ij")
    xi = np.zeros((A0.size, 3))
    xi[:, d] = 1.0 if s else -1.0
    xi[:, t[0]] = A0.ravel()
    xi[:, t[1]] = A1.ravel()
    return _map(mesh, e, xi)


# ------------------------------------------------------------------ states
def _conserved(rho, v1, v2, v3, p, gamma=GAMMA):
    rE = p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2 + v3 * v3)
    return [rho, rho * v1, rho * v2, rho * v3, rE]


def tgv_state(x, mach, gamma=GAMMA):
    """Taylor-Green vortex initial condition (T = 1, rho from the ideal gas)."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    v1 = np.sin(X) * np.cos(Y) * np.cos(Z)
    v2 = -np.cos(X) * np.sin(Y) * np.cos(Z)
    v3 = 0.0 * X
    p = 1.0 / (gamma * mach ** 2) + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    rho = gamma * mach ** 2 * p  # T = gamma M^2 p / rho = 1
    return np.stack(_conserved(rho, v1, v2, v3, p, gamma), axis=-1)


def bl_state(x, mach, ly, gamma=GAMMA):
    """Boundary-layer-like profile: rho = 1, T = 1, v1 = tanh(3 y / L_y)."""
    Y = x[..., 1]
    rho = 1.0 + 0.0 * Y
    v1 = np.tanh(3.0 * Y / ly)
    p = rho / (gamma * mach ** 2)
    zero = 0.0 * Y
    return np.stack(_conserved(rho, v1, zero, zero, p, gamma), axis=-1)


def _grad_complex_step(fn, x, h=1e-30):
    """d fn / d x_j by the complex-step rule; returns [..., 5, 3]."""
    out = []
    for j in range(3):
        xc = x.astype(complex)
        xc[..., j] += 1j * h
        out.append(np.imag(fn(xc)) / h)
    return np.stack(out, axis=-1)


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    mach: float
    reynolds: float
    gamma: float
    prandtl: float
    tau: float
    dt: float
    alpha: float
    visc_law: int          # 0 constant mu = 1, 1 nondimensional Sutherland
    Q: np.ndarray          # packed [sum_e 15 N_p]   layout [e][3c+j][node]
    U: np.ndarray          # packed [sum_e 5 N_p]    layout [e][c][node]
    Un: np.ndarray         # packed [sum_e 5 N_p]
    Uhat: np.ndarray       # packed [sum_F 5 N_fp]   layout [F][c][node]
    nu: np.ndarray         # packed [sum_e N_p]
    Ub: np.ndarray         # packed like Uhat; prescribed boundary state on boundary faces
    x: np.ndarray          # seeded unit-norm trace vector (matvec input)
    gmres_m: int
    seed: int


def make_state(mesh: Mesh, field, *, mach, reynolds=1600.0, noise=0.0, nu_amp=0.0,
               seed=0, name="custom", gmres_m=30, gamma=GAMMA, prandtl=PRANDTL, tau=TAU,
               dt=DT, alpha=None, visc_law=1, boundary_field=None) -> Workload:
    """Sample ``field(x) -> [..., 5]`` at nodes; add seeded noise.

    U = field + U(-noise, noise) per nodal value; Un = field (noise free);
    Q = grad field (complex step); Uhat = field at trace nodes + U(-noise, noise);
    nu = nu_amp * (1 + sin(x + f1) sin(y + f2) sin(z + f3)) with seeded phases.
    """
    ss = np.random.SeedSequence(seed)
    r_noise, r_hat, r_nu, r_x = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(4)]
    noff = mesh.node_offsets()
    foff = mesh.face_offsets()
    U = np.zeros(5 * noff[-1])
    Un = np.zeros(5 * noff[-1])
    Q = np.zeros(15 * noff[-1])
    nu = np.zeros(noff[-1])
    phases = r_nu.uniform(0.0, 2 * math.pi, size=3)
    for e in range(mesh.n_elem):
        xyz = element_node_xyz(mesh, e)
        npn = xyz.shape[0]
        u = field(xyz)                      # [N_p, 5]
        g = _grad_complex_step(field, xyz)  # [N_p, 5, 3]
        s5 = slice(5 * noff[e], 5 * noff[e] + 5 * npn)
        Un[s5] = u.T.ravel()
        U[s5] = u.T.ravel()
        Q[15 * noff[e]: 15 * noff[e] + 15 * npn] = g.reshape(npn, 15).T.ravel()
        if nu_amp > 0.0:
            nu[noff[e]: noff[e] + npn] = nu_amp * (1.0 + np.sin(xyz[:, 0] + phases[0])
                                                   * np.sin(xyz[:, 1] + phases[1])
                                                   * np.sin(xyz[:, 2] + phases[2]))
    if noise > 0.0:
        U += r_noise.uniform(-noise, noise, size=U.shape)
    Uhat = np.zeros(foff[-1])
    Ub = np.zeros(foff[-1])
    bfield = field if boundary_field is None else boundary_field
    for F in range(mesh.n_face):
        xyz = face_node_xyz(mesh, F)
        Uhat[foff[F]:foff[F + 1]] = field(xyz).T.ravel()
        if mesh.face_bc[F]:
            Ub[foff[F]:foff[F + 1]] = bfield(xyz).T.ravel()
    if noise > 0.0:
        Uhat += r_hat.uniform(-noise, noise, size=Uhat.shape)
    x = r_x.standard_normal(foff[-1])
    x /= np.linalg.norm(x)
    return Workload(name, mesh, mach, reynolds, gamma, prandtl, tau, dt,
                    dirk_alpha() if alpha is None else alpha, visc_law,
                    Q, U, Un, Uhat, nu, Ub, x, gmres_m, seed)


# ------------------------------------------------------------- the configs
def config(idx: int, *, n_override: Optional[int] = None) -> Workload:
    """The five synthetic workloads.

    0: 4^3 periodic TGV, p=2, M=0.1, noise 1e-3.
    1: 8^3 periodic supersonic TGV, p=3, M=1.25, smooth AV field in [0, 1e-3].
    2: same inputs as 1 (the mixed-precision run).
    3: 20x10x10 wall-stretched perturbed box, p drawn from {2,3,4}, M=0.5,
       elements numbered by degree (one contiguous range per degree).
    4: 12^3 periodic supersonic TGV, p=4, noise 1e-3.
    ``n_override`` shrinks the cube for quick tests (periodic configs only).
    """
    if idx == 0:
        n = n_override or 4
        mesh = box_mesh((n, n, n), p=2)
        return make_state(mesh, lambda x: tgv_state(x, 0.1), mach=0.1, noise=1e-3, seed=0,
                          name=f"tgv{n}^3-p2-M0.1", gmres_m=30)
    if idx in (1, 2):
        n = n_override or 8
        mesh = box_mesh((n, n, n), p=3)
        return make_state(mesh, lambda x: tgv_state(x, 1.25), mach=1.25, nu_amp=5e-4, seed=1,
                          name=f"tgv{n}^3-p3-M1.25-av", gmres_m=30)
    if idx == 3:
        nx, ny, nz = 20, 10, 10
        lx, lz = 2 * math.pi, math.pi
        h1 = (lx / nx) / 50.0
        yc = np.concatenate([[0.0], np.cumsum(h1 * 1.15 ** np.arange(ny))])
        ly = float(yc[-1])
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([3, 7])))
        pe = rng.choice([2, 3, 4], size=nx * ny * nz, p=[0.3, 0.5, 0.2])
        mesh = group_by_degree(box_mesh((nx, ny, nz), lengths=(lx, ly, lz), periodic=(True, False, True),
                                        y_coords=yc, perturb=0.02, p=pe, seed=3))
        f = lambda x: bl_state(x, 0.5, ly)
        return make_state(mesh, f, mach=0.5, noise=1e-3, seed=3, name="bl20x10x10-p234-M0.5",
                          gmres_m=30, boundary_field=f)
    if idx == 4:
        n = n_override or 12
        mesh = box_mesh((n, n, n), p=4)
        return make_state(mesh, lambda x: tgv_state(x, 1.25), mach=1.25, noise=1e-3, seed=4,
                          name=f"tgv{n}^3-p4-M1.25", gmres_m=50)
    raise ValueError(idx)
