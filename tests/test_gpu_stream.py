"""Streamed condensation (HDG_MIXED): one chunk of element systems at a time,
X = A^{-1}[B | R_qu] retained per element (hdg_store_x) and the interior
recovered from it (hdg_recover_interior_x).  The same kernels run on the same
data as with every system resident, so every output must be bit-identical:
the condensed systems, S, g, the GMRES history and increment, the recovered
interior increment, and whole Newton solves."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _equal(a, b):
    import torch
    return bool(torch.equal(a, b))


def test_streamed_step_matches_resident_step():
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth
    wl = synth.config(1)  # 8^3 periodic, p = 3 (512 elements)
    print("[stream] 8^3 p=3 mixed step, resident and streamed in chunks of 96", flush=True)
    res = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, chunk=96)
    stm = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, chunk=96, ctx=res.ctx, stream_E=True)
    ctx = res.ctx
    assert stm.E.numel() == int(ctx.layout["E_off"][96])  # one chunk of systems, not all of them
    res.run_calls()
    stm.run_calls()
    torch.cuda.synchronize()
    for name in ("SK", "S", "g", "hist", "dUhat", "dQU", "info"):
        assert _equal(getattr(res, name), getattr(stm, name)), name
    # the retained X is the X of the resident systems
    xo, eo = ctx.layout["x_off"], ctx.layout["E_off"]
    for e in (0, 95, 96, 311, 511):
        n, f = int(ctx.layout["elem_n"][e]), int(ctx.layout["elem_f"][e])
        ld = (int(eo[e + 1]) - int(eo[e])) // (n + f)
        xl = (int(xo[e + 1]) - int(xo[e])) // n
        Er = res.E[int(eo[e]):int(eo[e + 1])].view(n + f, ld)[:n, n:n + f + 1]
        Xs = stm.X[int(xo[e]):int(xo[e + 1])].view(n, xl)
        assert _equal(Xs[:, :f + 1], Er) and not Xs[:, f + 1:].any().item(), e
    print(f"  E resident {res.E.numel() * 8 / 1e9:.2f} GB, streamed {stm.E.numel() * 8 / 1e9:.2f} GB"
          f" + X {stm.X.numel() * 8 / 1e9:.2f} GB; dUhat, dQU identical")


def test_streamed_newton_solve_matches_resident():
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth
    mesh = synth.box_mesh((2, 2, 2), p=2, perturb=0.05, seed=5)
    wl = synth.make_state(mesh, lambda x: synth.tgv_state(x, 0.8), mach=0.8, noise=1e-2, seed=5, reynolds=400.0,
                          gmres_m=40)
    hists, states = [], []
    for stream_E in (False, True):
        print(f"[stream] Newton solve on a 2^3 p=2 mesh, chunks of 3, streamed={stream_E}", flush=True)
        st = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, chunk=3, stream_E=stream_E)
        h = pipeline.NewtonSolver(st, rb_max=4, maxit=3).solve()
        torch.cuda.synchronize()
        hists.append(h)
        states.append([t.clone() for t in (st.Q, st.U, st.Uhat)])
    assert len(hists[0]) == len(hists[1])
    for a, b in zip(hists[0], hists[1]):
        assert a[:4] == b[:4]
        assert (a[4] is None and b[4] is None) or np.array_equal(a[4], b[4])
    for a, b in zip(*states):
        assert _equal(a, b)
    print("  residual norms:", ["%.3e" % np.sqrt(sum(v * v for v in h[:3])) for h in hists[1]])


def test_store_and_recover_x_argument_errors():
    import ctypes
    from paper_2608_27863_amd import hdg, synth
    wl = synth.config(0)
    ctx = hdg.Context(wl.mesh, wl)
    L, h = ctx.L, ctx.h
    INVALID = -1  # HDG_ERR_INVALID_ARGUMENT
    dummy = ctypes.c_void_p(16)  # never dereferenced: every call below is rejected on the host
    assert L.hdg_store_x(h, -1, 1, dummy, dummy, None) == INVALID
    assert L.hdg_store_x(h, 0, ctx.n_elem + 1, dummy, dummy, None) == INVALID
    assert L.hdg_store_x(h, 0, 1, None, dummy, None) == INVALID
    assert L.hdg_store_x(h, 0, 1, dummy, None, None) == INVALID
    assert L.hdg_recover_interior_x(h, 0, 0, dummy, dummy, dummy, None) == INVALID
    assert L.hdg_recover_interior_x(h, 0, 1, None, dummy, dummy, None) == INVALID
    assert L.hdg_recover_interior_x(h, 0, 1, dummy, dummy, None, None) == INVALID
    ctx.close()
