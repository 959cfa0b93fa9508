"""CPU oracle of the artificial-viscosity field (TEST INFRASTRUCTURE ONLY).

Only ``tests/`` may import this module; it shares no code with the HIP path.
Written from eq. av-coeffs and the smoothing operator S_h (section 2.1), with
the readings the library documents for what the paper leaves open: the
compression -div v limited to [0, inf) as the divergence argument, the
vorticity limited to [0, inf), the sensor limited to [0, s_max], the acoustic
scale c* = sqrt(gamma p*/rho*) of the state with rho, p bounded below, the raw
elemental value = the maximum over the element's Gauss-Lobatto nodes, and
S_h = averaging element -> vertex (vertices shared through faces, periodic
pairs included) -> element, the final field being the trilinear interpolant
of the last vertex values.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def node_sensor(w, q, gamma, k, prm):
    """Sensor value c_av L(s) at one node from the state w (5) and its gradient
    q (15, q[3c+j] = du_c/dx_j)."""
    rho = w[0]
    v = np.array(w[1:4]) / rho
    p = (gamma - 1.0) * (w[4] - 0.5 * rho * (v @ v))
    G = np.zeros((3, 3))  # G[i, j] = dv_i/dx_j
    for i in range(3):
        for j in range(3):
            G[i, j] = (q[3 * (1 + i) + j] - v[i] * q[j]) / rho
    div = G[0, 0] + G[1, 1] + G[2, 2]
    curl = np.array([G[2, 1] - G[1, 2], G[0, 2] - G[2, 0], G[1, 0] - G[0, 1]])
    om = math.sqrt(curl @ curl)
    cstar = math.sqrt(gamma * max(p, prm["p_min"]) / max(rho, prm["rho_min"]))
    Ld = min(max(-div, 0.0), math.inf)
    Lw = min(max(om, 0.0), math.inf)
    s = math.sqrt(prm["h_m"] / k) * (Ld / cstar) * (Ld ** 2 / (Ld ** 2 + Lw ** 2 + prm["eps"]))
    return prm["c_av"] * min(max(s, 0.0), prm["s_max"])


def raw_elemental(wl, U, Q, prm):
    sz = O.Sizes(wl.mesh)
    out = np.zeros(wl.mesh.n_elem)
    for e in range(wl.mesh.n_elem):
        Np = sz.Np(e)
        o = sz.noff[e]
        u = U[5 * o:5 * (o + Np)].reshape(5, Np)
        q = Q[15 * o:15 * (o + Np)].reshape(15, Np)
        k = int(wl.mesh.elem_p[e])
        out[e] = max(node_sensor(u[:, i], q[:, i], wl.gamma, k, prm) for i in range(Np))
    return out


def vertex_classes(mesh):
    """Classes of vertices identified through every two-sided face: corner c of
    the side-0 element on local face l0 matches the corner of the side-1
    element with the same position along the face's two tangential axes."""
    label = list(range(mesh.n_vert))

    def find(a):
        path = []
        while label[a] != a:
            path.append(a)
            a = label[a]
        for b in path:
            label[b] = a
        return a

    for F in range(mesh.n_face):
        (e0, l0), (e1, l1) = mesh.face_elem[F]
        if e1 < 0:
            continue
        d = l0 // 2
        for c in range(8):
            if (c >> d) & 1 != l0 % 2:
                continue
            c1 = (c & ~(1 << d)) | ((l1 % 2) << d)
            a, b = find(int(mesh.elem_vert[e0, c])), find(int(mesh.elem_vert[e1, c1]))
            if a != b:
                label[max(a, b)] = min(a, b)
    return np.array([[find(int(mesh.elem_vert[e, c])) for c in range(8)] for e in range(mesh.n_elem)])


def smooth(mesh, raw, iters):
    """S_h: `iters` element->vertex averagings with vertex->element averagings
    in between; returns the vertex values (dict class -> value) and the corner
    classes."""
    cls = vertex_classes(mesh)
    elem = np.array(raw, dtype=np.float64)
    vert = {}
    for it in range(iters):
        acc, cnt = {}, {}
        for e in range(mesh.n_elem):
            for c in range(8):
                acc[cls[e, c]] = acc.get(cls[e, c], 0.0) + elem[e]
                cnt[cls[e, c]] = cnt.get(cls[e, c], 0) + 1
        vert = {k: acc[k] / cnt[k] for k in acc}
        if it + 1 < iters:
            elem = np.array([np.mean([vert[cls[e, c]] for c in range(8)]) for e in range(mesh.n_elem)])
    return vert, cls


def av_field(wl, U, Q, prm, iters):
    """Nodal artificial viscosity (packed node array) and the raw elemental values."""
    raw = raw_elemental(wl, U, Q, prm)
    m = wl.mesh
    sz = O.Sizes(m)
    nu = np.zeros(int(sz.noff[-1]))
    if iters == 0:
        for e in range(m.n_elem):
            nu[sz.noff[e]:sz.noff[e + 1]] = raw[e]
        return nu, raw
    vert, cls = smooth(m, raw, iters)
    for e in range(m.n_elem):
        p = int(m.elem_p[e])
        r = O.gll(p)
        vals = []
        for i2 in range(p + 1):
            for i1 in range(p + 1):
                for i0 in range(p + 1):
                    xi = (r[i0], r[i1], r[i2])
                    t = 0.0
                    for c in range(8):
                        wgt = 1.0
                        for d in range(3):
                            wgt *= 0.5 * (1 + xi[d]) if (c >> d) & 1 else 0.5 * (1 - xi[d])
                        t += wgt * vert[cls[e, c]]
                    vals.append(t)
        nu[sz.noff[e]:sz.noff[e + 1]] = vals
    return nu, raw
