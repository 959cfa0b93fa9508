"""CPU oracle of the solver loop around the hot path (TEST INFRASTRUCTURE ONLY).

Only ``tests/`` may import this module.  It shares no code with the HIP path
and builds on ``oracle.py`` (element systems, condensation, trace system,
GMRES, recovery).  Written from the paper:

* the reduced-basis initial guess (section 3.4, eq. rb-min): the least-squares
  problem min ||g - Z c||_2 over the stored projected vectors, x0 = W c, and the
  first-in first-out window of accepted corrections, one new product S w per
  accepted solve;
* Newton's method on the stage residual (section 2.4, eqs. nonlinear-residual,
  newton-linearization, newton-update) with static condensation inside each
  iteration (section 2.5) and the residual norm as the convergence measure;
* the diagonally implicit Runge-Kutta stages and update (section 2.3,
  eqs. dirk-stage, dirk-update) with the three-stage, third-order L-stable
  tableau of Alexander.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


# ------------------------------------------------------------ reduced basis
def rb_guess(W, Z, g):
    """eq. rb-min: c = argmin ||g - Z c||_2 (least squares, library routine),
    x0 = W c.  W, Z are N x nb (nb may be 0)."""
    if W.shape[1] == 0:
        return np.zeros(g.shape[0]), np.zeros(0)
    c, *_ = np.linalg.lstsq(Z, g, rcond=None)
    return W @ c, c


class RBWindow:
    """Fixed window of the nb_max most recent accepted corrections w and their
    products z = S w: inserting into a full window discards the oldest pair."""

    def __init__(self, nb_max):
        self.nb_max = int(nb_max)
        self.ws, self.zs = [], []

    def insert(self, w, z):
        self.ws.append(np.array(w, dtype=np.float64))
        self.zs.append(np.array(z, dtype=np.float64))
        if len(self.ws) > self.nb_max:
            self.ws.pop(0)
            self.zs.pop(0)

    def arrays(self, N):
        if not self.ws:
            return np.zeros((N, 0)), np.zeros((N, 0))
        return np.stack(self.ws, axis=1), np.stack(self.zs, axis=1)


# --------------------------------------------------------------------- DIRK
def alexander_tableau():
    """Three-stage, third-order, L-stable DIRK of Alexander: gamma is the root in
    (0, 1) of x^3 - 3x^2 + 3x/2 - 1/6 near 0.4359; tau2 = (1 + gamma)/2;
    b1 = -(6 gamma^2 - 16 gamma + 1)/4, b2 = (6 gamma^2 - 20 gamma + 5)/4,
    b3 = gamma, and the last row of A equals b (stiffly accurate)."""
    roots = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
    gam = float(min((r.real for r in roots if abs(r.imag) < 1e-12 and 0.3 < r.real < 0.5)))
    t2 = 0.5 * (1.0 + gam)
    b1 = -(6.0 * gam ** 2 - 16.0 * gam + 1.0) / 4.0
    b2 = (6.0 * gam ** 2 - 20.0 * gam + 5.0) / 4.0
    A = np.array([[gam, 0.0, 0.0], [t2 - gam, gam, 0.0], [b1, b2, gam]])
    b = np.array([b1, b2, gam])
    c = np.array([gam, t2, 1.0])
    return A, b, c


def dirk_coefficients(A, b):
    """d = A^{-1} (entries d_ij) and e_j = sum_i b_i d_ij (eqs. dirk-stage,
    dirk-update)."""
    d = np.linalg.inv(A)
    return d, b @ d


def lagged_state(d, i, Un, stages):
    """The stage-i mass term sum_{j<=i} d_ij M (U^{n,j} - U^n) written as
    d_ii M (U^{n,i} - Ut) with Ut = U^n - sum_{j<i} (d_ij / d_ii)(U^{n,j} - U^n)."""
    Ut = np.array(Un, dtype=np.float64)
    for j in range(i):
        Ut = Ut - (d[i, j] / d[i, i]) * (stages[j] - Un)
    return Ut


def dirk_update(e, Un, stages):
    """eq. dirk-update: U^{n+1} = (1 - sum_j e_j) U^n + sum_j e_j U^{n,j}."""
    out = (1.0 - float(np.sum(e))) * np.array(Un, dtype=np.float64)
    for j, Uj in enumerate(stages):
        out = out + e[j] * Uj
    return out


# ------------------------------------------------------------------- Newton
def residual_norms(wl, sz, Es):
    """(||R_q||, ||R_u||, ||R_uh||) of the stage residual (eq. nonlinear-residual)
    from the residual columns of the element systems; R_uh is the assembled
    trace residual sum_K P_K^T R_uh^K (eq. trace-residual)."""
    m = wl.mesh
    rq = ru = 0.0
    Rh = np.zeros(int(sz.foff[-1]))
    for e, E in enumerate(Es):
        n = sz.n(e)
        Np = n // 20
        r = E[:, -1]
        rq += float(np.sum(r[:15 * Np] ** 2))
        ru += float(np.sum(r[15 * Np:n] ** 2))
        t = np.concatenate([[0], np.cumsum(sz.face_sizes(e))])
        for a, F in enumerate(m.elem_face[e]):
            Rh[sz.foff[F]:sz.foff[F + 1]] += r[n + t[a]:n + t[a + 1]]
    return math.sqrt(rq), math.sqrt(ru), float(np.linalg.norm(Rh))


def admissible(wl, U, dU, alpha):
    """U + alpha dU has positive density and pressure at every node."""
    sz = O.Sizes(wl.mesh)
    for e in range(wl.mesh.n_elem):
        Np = sz.Np(e)
        o = sz.noff[e]
        w = (U[5 * o:5 * (o + Np)] + alpha * dU[5 * o:5 * (o + Np)]).reshape(5, Np)
        rho = w[0]
        p = (wl.gamma - 1.0) * (w[4] - 0.5 * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2) / rho)
        if not (np.all(rho > 0.0) and np.all(p > 0.0) and np.all(np.isfinite(p))):
            return False
    return True


def newton_solve(wl, Q, U, Uhat, m, tol=1e-10, maxit=8, rb=None, gmres_tol=0.0, gmres_restarts=1, atol=1e-11):
    """Newton's method for the stage residual with the lagged state wl.Un.
    Iteration k: element systems at W^k; stop once
    ||F(W^k)|| <= max(atol, tol ||F(W^0)||);
    else condensation, the reduced-basis guess (if a window is given),
    left-preconditioned GMRES(m) on S dUhat = g from it, recovery, and the
    update W^{k+1} = W^k + alpha dW with alpha = 1 halved until the state is
    admissible.  Accepted corrections enter the window.  Returns the state and
    the history [(||R_q||, ||R_u||, ||R_uh||, alpha, gmres_hist), ...]."""
    sz = O.Sizes(wl.mesh)
    Q, U, Uhat = (np.array(a, dtype=np.float64) for a in (Q, U, Uhat))
    hist = []
    f0 = None
    for it in range(maxit + 1):
        Es = [np.array(O.element_system(wl, e, sz, U=U, Q=Q, Uhat=Uhat)) for e in range(wl.mesh.n_elem)]
        nr = residual_norms(wl, sz, Es)
        fn = math.sqrt(sum(v * v for v in nr))
        f0 = fn if f0 is None else f0
        if fn <= max(atol, tol * f0) or it == maxit:
            hist.append((*nr, None, None))
            break
        outs = [O.condense(E, sz.n(e)) for e, E in enumerate(Es)]
        ts = O.TraceSystem(wl, [o[0] for o in outs], [o[1] for o in outs])
        x0 = None
        if rb is not None and rb.ws:
            Wm, Zm = rb.arrays(ts.N)
            x0, _ = rb_guess(Wm, Zm, ts.g)
        dUh, gh = O.gmres(ts, ts.g, m, tol=gmres_tol, x0=x0, restarts=gmres_restarts)
        if rb is not None:
            rb.insert(dUh, ts.matvec(dUh))
        dQU = np.concatenate([O.recover(wl, sz, e, outs[e][2], dUh) for e in range(wl.mesh.n_elem)])
        dQ, dU = _split_dqu(sz, wl.mesh.n_elem, dQU)
        alpha = 1.0
        while not admissible(wl, U, dU, alpha) and alpha > 2.0 ** -10:
            alpha *= 0.5
        Q = Q + alpha * dQ
        U = U + alpha * dU
        Uhat = Uhat + alpha * dUh
        hist.append((*nr, alpha, gh))
    return Q, U, Uhat, hist


def _split_dqu(sz, ne, dQU):
    """Packed [e][20][node] increments -> (dQ [e][15][node], dU [e][5][node])."""
    dQ, dU = [], []
    for e in range(ne):
        Np = sz.Np(e)
        o = 20 * sz.noff[e]
        dQ.append(dQU[o:o + 15 * Np])
        dU.append(dQU[o + 15 * Np:o + 20 * Np])
    return np.concatenate(dQ), np.concatenate(dU)


def dirk_step(wl, Q, U, Uhat, m, tol=1e-10, maxit=8, rb=None, gmres_tol=0.0, gmres_restarts=1, atol=1e-11):
    """One time step of the three-stage DIRK (eqs. dirk-stage, dirk-update):
    stage i solves the HDG system with the mass term lagged on
    Ut_i = U^n - sum_{j<i} (d_ij/d_ii)(U^{n,j} - U^n), starting from the previous
    stage's converged state (stage 1 from W^n); then U^{n+1} by eq. dirk-update,
    with Q and Uhat of the last stage (the tableau is stiffly accurate, so the
    last stage is the step's end state).  wl.alpha must equal d_ii.  Returns
    the new state and the per-stage Newton histories."""
    A, b, _ = alexander_tableau()
    d, e = dirk_coefficients(A, b)
    assert abs(wl.alpha - d[0, 0]) < 1e-12 * d[0, 0]
    Un = np.array(U, dtype=np.float64)
    stages, hists = [], []
    Un_saved = wl.Un
    try:
        for i in range(3):
            wl.Un = lagged_state(d, i, Un, stages)
            Q, U, Uhat, h = newton_solve(wl, Q, U, Uhat, m, tol=tol, maxit=maxit, rb=rb, gmres_tol=gmres_tol,
                                         gmres_restarts=gmres_restarts, atol=atol)
            stages.append(U.copy())
            hists.append(h)
    finally:
        wl.Un = Un_saved
    return Q, dirk_update(e, Un, stages), Uhat, hists
