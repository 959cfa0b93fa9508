"""Pins of the solver-loop oracle (oracle/newton.py) against facts fixed by
the paper and by mathematics:

* the DIRK tableau: the order conditions of a third-order method, stiff
  accuracy and L-stability (the stability function vanishes at infinity);
* the stage algebra of eqs. dirk-stage and dirk-update, run on the scalar
  test equation y' = lambda y, reproduces the stability function
  R(z) = 1 + z b^T (I - z A)^{-1} 1 computed from the Butcher form;
* the reduced-basis guess of eq. rb-min: exact when g lies in span(Z) with
  Z = S W, the residual orthogonal to span(Z), duplicated columns change
  nothing, first-in first-out window semantics;
* Newton's method: a uniform state is a solution (converged before any
  iteration, and unchanged by a whole DIRK step); a perturbed state converges
  quadratically; a DIRK step on a periodic mesh conserves the integral of
  every conserved variable (sum of eq. hdg-cons over elements with the
  single-valued trace flux).
"""
import math

import numpy as np
import pytest

from paper_2608_27863_amd import synth
from oracle import newton as N
from oracle import oracle as O


def test_tableau_order_and_l_stability():
    A, b, c = N.alexander_tableau()
    one = np.ones(3)
    assert np.allclose(A @ one, c, atol=1e-15)
    assert abs(b.sum() - 1.0) < 1e-15                    # order 1
    assert abs(b @ c - 0.5) < 1e-15                      # order 2
    assert abs(b @ c ** 2 - 1.0 / 3.0) < 1e-14           # order 3
    assert abs(b @ A @ c - 1.0 / 6.0) < 1e-14
    assert np.allclose(A[2], b, atol=0)                  # stiffly accurate
    g = A[0, 0]
    assert abs(g ** 3 - 3 * g ** 2 + 1.5 * g - 1.0 / 6.0) < 1e-15
    assert abs(1.0 / g - synth.dirk_alpha()) < 1e-12 * synth.dirk_alpha()
    R = lambda z: 1.0 + z * b @ np.linalg.solve(np.eye(3) - z * A, one)
    assert abs(R(-1e12)) < 1e-10                         # L-stable: R(-inf) = 0
    for y in np.linspace(-50, 50, 41):
        assert abs(R(1j * y)) <= 1.0 + 1e-13             # A-stable on the imaginary axis
    # the fourth-order condition fails (the method is exactly third order)
    assert abs(b @ c ** 3 - 0.25) > 1e-3


@pytest.mark.parametrize("lam_dt", [-0.3, -5.0, 2.0, -40.0])
def test_stage_algebra_reproduces_the_stability_function(lam_dt):
    """y' = lambda y in the form of eq. dirk-stage with M = 1 and
    N(y) = -lambda y: d_ii (Y_i - Ut_i) - dt lambda Y_i = 0 per stage, with the
    oracle's lagged state Ut_i and update."""
    A, b, c = N.alexander_tableau()
    d, e = N.dirk_coefficients(A, b)
    yn = np.array([1.3])
    stages = []
    for i in range(3):
        Ut = N.lagged_state(d, i, yn, stages)
        stages.append(d[i, i] * Ut / (d[i, i] - lam_dt))
    y1 = N.dirk_update(e, yn, stages)
    R = 1.0 + lam_dt * b @ np.linalg.solve(np.eye(3) - lam_dt * A, np.ones(3))
    assert abs(y1[0] - R * yn[0]) < 1e-13 * abs(yn[0]), (y1, R * yn)


def test_lagged_state_against_the_stage_sum():
    """d_ii (U_i - Ut_i) equals sum_{j<=i} d_ij (U_j - U^n) for any vectors."""
    rng = np.random.default_rng(4)
    A, b, _ = N.alexander_tableau()
    d, _ = N.dirk_coefficients(A, b)
    Un = rng.standard_normal(7)
    stages = [rng.standard_normal(7) for _ in range(3)]
    for i in range(3):
        Ut = N.lagged_state(d, i, Un, stages[:i])
        lhs = d[i, i] * (stages[i] - Ut)
        rhs = sum(d[i, j] * (stages[j] - Un) for j in range(i + 1))
        assert np.allclose(lhs, rhs, rtol=0, atol=1e-13)


def _rb_problem(N_=400, nb=6, seed=0):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((N_, N_)) / math.sqrt(N_) + 3.0 * np.eye(N_)
    W = rng.standard_normal((N_, nb))
    return rng, S, W, S @ W


def test_rb_guess_exact_in_span_and_optimal():
    rng, S, W, Z = _rb_problem()
    c_true = rng.standard_normal(W.shape[1])
    g = Z @ c_true
    x0, c = N.rb_guess(W, Z, g)
    assert np.allclose(c, c_true, rtol=0, atol=1e-12)
    assert np.linalg.norm(S @ x0 - g) < 1e-12 * np.linalg.norm(g)      # the exact solution of S x = g
    g2 = g + rng.standard_normal(g.shape[0])
    x0, c = N.rb_guess(W, Z, g2)
    r = g2 - Z @ c
    assert np.abs(Z.T @ r).max() < 1e-10 * np.linalg.norm(Z) * np.linalg.norm(g2)   # normal equations
    # duplicated (w, z) pairs leave the guess unchanged
    x_dup, _ = N.rb_guess(np.concatenate([W, W[:, :2]], 1), np.concatenate([Z, Z[:, :2]], 1), g2)
    assert np.linalg.norm(x_dup - x0) < 1e-10 * np.linalg.norm(x0)
    # empty window: zero guess
    x_e, _ = N.rb_guess(W[:, :0], Z[:, :0], g2)
    assert not np.any(x_e)


def test_rb_window_is_first_in_first_out():
    win = N.RBWindow(3)
    for k in range(5):
        win.insert(np.full(4, float(k)), np.full(4, 10.0 + k))
    Wm, Zm = win.arrays(4)
    assert Wm.shape == (4, 3)
    assert np.array_equal(Wm[0], [2.0, 3.0, 4.0]) and np.array_equal(Zm[0], [12.0, 13.0, 14.0])


def _small(p=1, n=2, noise=2e-3, seed=6, mach=0.5):
    mesh = synth.box_mesh((n, n, n), p=p, perturb=0.1, seed=seed)
    return synth.make_state(mesh, lambda x: synth.tgv_state(x, mach), mach=mach, noise=noise, seed=seed,
                            reynolds=200.0, gmres_m=40)


def test_uniform_state_is_a_solution():
    const = np.array(synth._conserved(1.1, 0.3, -0.2, 0.1, 0.9))
    field = lambda x: np.broadcast_to(const, x.shape[:-1] + (5,)) + 0.0 * x[..., :1]
    mesh = synth.box_mesh((2, 2, 2), p=1, perturb=0.1, seed=2)
    wl = synth.make_state(mesh, field, mach=0.5, noise=0.0, seed=2)
    wl.Q[:] = 0.0
    sz = O.Sizes(mesh)
    Es = [np.array(O.element_system(wl, e, sz)) for e in range(mesh.n_elem)]
    assert max(N.residual_norms(wl, sz, Es)) < 1e-12
    Q, U, Uh, hists = N.dirk_step(wl, wl.Q, wl.U, wl.Uhat, m=20)
    assert all(len(h) == 1 for h in hists)          # every stage converged before iterating
    assert np.array_equal(U, wl.U) and np.array_equal(Uh, wl.Uhat) and np.array_equal(Q, wl.Q)


def test_newton_converges_quadratically():
    wl = _small(noise=5e-2)
    Q, U, Uh, hist = N.newton_solve(wl, wl.Q, wl.U, wl.Uhat, m=60, tol=1e-13, maxit=6, gmres_tol=1e-14,
                                    gmres_restarts=4)
    f = [math.sqrt(h[0] ** 2 + h[1] ** 2 + h[2] ** 2) for h in hist]
    assert all(h[3] == 1.0 for h in hist[:-1])      # full steps
    assert f[-1] <= 1e-13 * f[0], f
    # quadratic: f_{k+1} / f_k^2 bounded while above rounding
    ratios = [f[k + 1] / f[k] ** 2 for k in range(len(f) - 1) if f[k + 1] > 1e-12 * f[0]]
    assert len(ratios) >= 2 and max(ratios[1:]) <= 10.0 * ratios[0] + 1e-300, (f, ratios)
    assert f[2] / f[1] < 0.1 * f[1] / f[0]          # faster than linear


def test_dirk_step_conserves_every_variable():
    wl = _small(p=1)
    sz = O.Sizes(wl.mesh)

    def totals(U):
        tot = np.zeros(5)
        for e in range(wl.mesh.n_elem):
            E = O.element_system(wl, e, sz)
            Np = sz.Np(e)
            M = E[:Np, :Np]
            o = sz.noff[e]
            tot += (M @ U[5 * o:5 * (o + Np)].reshape(5, Np).T).sum(axis=0)
        return tot

    t0 = totals(wl.U)
    Q, U1, Uh, hists = N.dirk_step(wl, wl.Q, wl.U, wl.Uhat, m=60, tol=1e-12, maxit=8, gmres_tol=1e-14,
                                   gmres_restarts=4)
    t1 = totals(U1)
    assert np.allclose(t1, t0, rtol=0, atol=1e-10 * np.abs(t0).max()), (t0, t1)
    assert np.linalg.norm(U1 - wl.U) > 1e-6 * np.linalg.norm(wl.U)  # the state did change
    assert all(len(h) >= 2 for h in hists)
