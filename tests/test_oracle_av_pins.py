"""Pins of the artificial-viscosity oracle (oracle/av.py) against closed forms
of eq. av-coeffs and properties of the smoothing operator S_h:

* a divergence-free velocity (the Taylor-Green initial field, a rigid
  rotation) and an expansion give no viscosity;
* a uniform compression v = -a x gives c_av sqrt(h/k) (3a / c) 9a^2/(9a^2 + eps);
  adding a rotation Omega x x lowers it by the Ducros factor with
  |curl v| = 2 |Omega|; the upper bound s_max clips it;
* smoothing a constant field returns the constant; the smoothed field lies
  between the raw extremes and is continuous across every face (periodic
  pairs included); vertex classes count n^3 on a periodic n^3 mesh.
"""
import math

import numpy as np
import pytest

from paper_2608_27863_amd import synth
from oracle import av as AV
from oracle import oracle as O

PRM = dict(c_av=2e-3, h_m=2 * math.pi / 8, eps=1e-10, s_max=math.inf, rho_min=1e-8, p_min=1e-8)


def _state(rho, v, p, G, gamma=1.4):
    """w, q at a point with uniform rho and p and velocity gradient G[i, j] = dv_i/dx_j."""
    v = np.asarray(v, float)
    w = np.array([rho, *(rho * v), p / (gamma - 1) + 0.5 * rho * v @ v])
    q = np.zeros((5, 3))
    for i in range(3):
        q[1 + i] = rho * G[i]
    q[4] = rho * (v @ G)
    return w, q.ravel()


def test_compression_closed_form_and_ducros_factor():
    rho, p, a, k = 1.2, 0.7, 0.8, 3
    c = math.sqrt(1.4 * p / rho)
    w, q = _state(rho, [0.1, -0.2, 0.3], p, -a * np.eye(3))
    got = AV.node_sensor(w, q, 1.4, k, PRM)
    want = PRM["c_av"] * math.sqrt(PRM["h_m"] / k) * (3 * a / c) * (9 * a * a) / (9 * a * a + PRM["eps"])
    assert abs(got - want) < 1e-15 * want
    Om = np.array([0.3, -0.4, 0.5])
    R = np.array([[0, -Om[2], Om[1]], [Om[2], 0, -Om[0]], [-Om[1], Om[0], 0]])  # v = Om x x
    w, q = _state(rho, [0.1, -0.2, 0.3], p, R - a * np.eye(3))
    got = AV.node_sensor(w, q, 1.4, k, PRM)
    want_d = PRM["c_av"] * math.sqrt(PRM["h_m"] / k) * (3 * a / c) * (9 * a * a) / (
        9 * a * a + 4 * Om @ Om + PRM["eps"])
    assert abs(got - want_d) < 1e-15 * want_d and got < want
    clipped = dict(PRM, s_max=1e-3)
    assert abs(AV.node_sensor(w, q, 1.4, k, clipped) - PRM["c_av"] * 1e-3) < 1e-18
    # expansion and pure rotation: no viscosity
    w, q = _state(rho, [0.1, -0.2, 0.3], p, +a * np.eye(3))
    assert AV.node_sensor(w, q, 1.4, k, PRM) == 0.0
    w, q = _state(rho, [0.1, -0.2, 0.3], p, R)
    assert AV.node_sensor(w, q, 1.4, k, PRM) < 1e-30


def test_taylor_green_initial_field_is_not_sensed():
    mesh = synth.box_mesh((3, 3, 3), p=2)
    wl = synth.make_state(mesh, lambda x: synth.tgv_state(x, 1.25), mach=1.25, noise=0.0, seed=1)
    raw = AV.raw_elemental(wl, wl.U, wl.Q, PRM)
    assert raw.max() < 1e-18


def _compressive(n=3, p=2, periodic=(True, True, True), seed=2):
    L = (2 * math.pi, 2 * math.pi if periodic[1] else 1.0, 2 * math.pi)
    mesh = synth.box_mesh((n, n, n), lengths=L, periodic=periodic, p=p, perturb=0.1, seed=seed)

    def field(x):
        u = synth.tgv_state(x, 1.25)
        rho = u[..., 0]
        v1 = u[..., 1] / rho + 0.4 * np.sin(x[..., 0])  # a compressive wave in x
        pr = 0.4 * (u[..., 4] - 0.5 * (u[..., 1] ** 2 + u[..., 2] ** 2 + u[..., 3] ** 2) / rho)
        return np.stack(synth._conserved(rho, v1, u[..., 2] / rho, u[..., 3] / rho, pr), axis=-1)

    return synth.make_state(mesh, field, mach=1.25, noise=0.0, seed=seed)


def test_smoothing_constant_bounds_and_continuity():
    wl = _compressive()
    m = wl.mesh
    sz = O.Sizes(m)
    raw = AV.raw_elemental(wl, wl.U, wl.Q, PRM)
    assert raw.max() > 0.0 and raw.min() >= 0.0
    vert, cls = AV.smooth(m, np.full(m.n_elem, 3.5e-4), 2)
    assert all(abs(v - 3.5e-4) < 1e-19 for v in vert.values())
    nu, raw2 = AV.av_field(wl, wl.U, wl.Q, PRM, 2)
    assert np.array_equal(raw, raw2)
    assert nu.min() >= raw.min() - 1e-18 and nu.max() <= raw.max() + 1e-18
    # continuity: the nodes of each face seen from its two elements carry the same values
    for F in range(m.n_face):
        (e0, l0), (e1, l1) = m.face_elem[F]
        if e1 < 0:
            continue
        vals = []
        for e, lf in ((e0, l0), (e1, l1)):
            p = int(m.elem_p[e])
            a = nu[sz.noff[e]:sz.noff[e + 1]].reshape(p + 1, p + 1, p + 1)  # [i2][i1][i0]
            d, side = lf // 2, lf % 2
            idx = [slice(None)] * 3
            idx[2 - d] = p if side else 0
            vals.append(a[tuple(idx)])
        assert np.allclose(vals[0], vals[1], rtol=0, atol=1e-18 + 1e-14 * raw.max())


@pytest.mark.parametrize("periodic,count", [((True, True, True), 27), ((True, False, True), 36)])
def test_vertex_classes(periodic, count):
    mesh = synth.box_mesh((3, 3, 3), lengths=(1.0, 1.0, 1.0), periodic=periodic, p=1)
    cls = AV.vertex_classes(mesh)
    assert len(set(cls.ravel().tolist())) == count
