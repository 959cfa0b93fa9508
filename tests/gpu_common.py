"""Shared helpers of the GPU parity tests: run the HIP path, extract results
into the documented layouts, compare with the oracle."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402

# FP64 path vs oracle: relative (Frobenius / 2-norm) error bound.
RTOL_FP64 = 1e-12


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(got - ref)
    return num / den if den > 0 else num


def assert_rel(got, ref, rtol, what):
    e = rel_err(got, ref)
    print(f"  {what}: rel err {e:.3e}", flush=True)
    assert e <= rtol, f"{what}: relative error {e:.3e} > {rtol:.1e}"
    return e


def e_view(ctx, Ehost, e, e0=0):
    """Element e's system as [n+f, n+f+1] from a host copy of a chunk starting at e0."""
    n = int(ctx.layout["elem_n"][e])
    f = int(ctx.layout["elem_f"][e])
    o = ctx.layout["E_off"]
    a = Ehost[int(o[e] - o[e0]):int(o[e + 1] - o[e0])]
    ld = a.size // (n + f)
    return a.reshape(n + f, ld)[:, :n + f + 1], ld


def sk_view(ctx, SKhost, e):
    f = int(ctx.layout["elem_f"][e])
    o = ctx.layout["SK_off"]
    m = SKhost[int(o[e]):int(o[e + 1])].reshape(f + 1, f).T
    return m[:, :f], m[:, f]


def bsr_blocks(ctx, Shost):
    """{(F, G): dense block} from the GPU block-sparse operator."""
    rp, col, vo, fo = (ctx.layout[k] for k in ("bsr_row_ptr", "bsr_col", "bsr_val_off", "face_off"))
    out = {}
    for F in range(ctx.n_face):
        bF = int(fo[F + 1] - fo[F])
        for k in range(int(rp[F]), int(rp[F + 1])):
            G = int(col[k])
            bG = int(fo[G + 1] - fo[G])
            out[(F, G)] = Shost[int(vo[k]):int(vo[k]) + bF * bG].reshape(bG, bF).T
    return out


def oracle_condensed(wl, elems=None, threads=None):
    """Oracle element systems and condensation for the given elements."""
    from concurrent.futures import ThreadPoolExecutor
    sz = O.Sizes(wl.mesh)
    elems = list(range(wl.mesh.n_elem)) if elems is None else list(elems)

    def one(e):
        E = O.element_system(wl, e, sz)
        SK, gK, X = O.condense(E, sz.n(e))
        return e, np.array(E), SK, gK, X

    with ThreadPoolExecutor(max_workers=threads or min(16, os.cpu_count() or 1)) as ex:
        res = list(ex.map(one, elems))
    return {e: dict(E=E, SK=SK, gK=gK, X=X) for e, E, SK, gK, X in res}


def residual_scale(wl, ctx, e, Eo):
    """Magnitude of the summands of the residual columns of element e:
    |[A B; C D]| |(W, Uhat^K)| (the residual is, to first order, this Jacobian
    applied to the state).  Rounding differences of two correct evaluations of
    the residual are bounded relative to it, not to the (cancelling) result."""
    sz = O.Sizes(wl.mesh)
    Np = sz.Np(e)
    o = sz.noff[e]
    w = np.concatenate([wl.Q[15 * o:15 * (o + Np)], wl.U[5 * o:5 * (o + Np)],
                        O.gather_trace(wl, sz, e, wl.Uhat)])
    n, f = sz.n(e), sz.f(e)
    J = np.abs(Eo[:, :n + f])
    return J @ np.abs(w)


def assembled_g_scale(wl, gKs):
    """sum_K |g^K| per trace entry: the assembled g is a sum of element terms
    that largely cancel on interior faces."""
    sz = O.Sizes(wl.mesh)
    out = np.zeros(int(sz.foff[-1]))
    for e, gK in enumerate(gKs):
        t = np.concatenate([[0], np.cumsum(sz.face_sizes(e))])
        for a, F in enumerate(wl.mesh.elem_face[e]):
            out[sz.foff[F]:sz.foff[F + 1]] += np.abs(gK[t[a]:t[a + 1]])
    return out


def recovery_checks(wl, e, Eo, X, dUhat, got):
    """(backward error / (n u), forward error / bound) of a recovered d(Q,U)^K.

    Backward: || A dW + B dUh^K + R_qu || / (||A|| ||dW|| + ||B|| ||dUh^K|| + ||R_qu||),
    at the level of u for any backward-stable solve (first block row of
    eq. newton-local-block).  Forward: the difference from the oracle's
    -(x_r + X_B dUh^K) relative to its bound 4 cond_2(A) u (|x_r| + |X_B||dUh^K|)."""
    sz = O.Sizes(wl.mesh)
    n = sz.n(e)
    A, B, C, D, Rq, Ru = O.split(Eo, n)
    d = O.gather_trace(wl, sz, e, dUhat)
    res = A @ got + B @ d + Rq
    back = np.linalg.norm(res) / (np.linalg.norm(A, 2) * np.linalg.norm(got) + np.linalg.norm(B, 2) *
                                  np.linalg.norm(d) + np.linalg.norm(Rq))
    f = d.shape[0]
    ref = -(X[:, f] + X[:, :f] @ d)
    scale = np.linalg.norm(np.abs(X[:, f]) + np.abs(X[:, :f]) @ np.abs(d))
    bound = 4.0 * np.linalg.cond(A) * np.finfo(np.float64).eps * scale
    # backward error reported as a fraction of n u (the textbook bound for LU solves)
    return back / (n * np.finfo(np.float64).eps), np.linalg.norm(got - ref) / bound


def recovery_error(wl, e, X, dUhat, got):
    """|| got - ref || relative to the summands of ref = -(x_r + X_B dUh^K):
    the two terms are O(1) and largely cancel, and each side carries the
    cond(A) u error of its own solve with A."""
    sz = O.Sizes(wl.mesh)
    d = O.gather_trace(wl, sz, e, dUhat)
    f = d.shape[0]
    ref = -(X[:, f] + X[:, :f] @ d)
    scale = np.abs(X[:, f]) + np.abs(X[:, :f]) @ np.abs(d)
    return np.linalg.norm(got - ref) / np.linalg.norm(scale), rel_err(got, ref)
