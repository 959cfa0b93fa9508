"""A whole Newton step captured in a HIP graph by the library
(hdg_graph_capture_newton, through the C ABI): every replay must reproduce the
eager step bit for bit, with the program's own eager work and
synchronisations between replays, on the default stream and on another one,
and must follow new contents of the input buffers.  The one-call step
(hdg_newton_step) must equal the step issued call by call."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

OUTS = ("E", "SK", "S", "g", "Sinv", "dUhat", "hist", "dQU")


def _outputs(st):
    return {k: getattr(st, k).cpu().numpy().copy() for k in OUTS}


@pytest.mark.parametrize("mixed", [False, True])
def test_graph_replays_match_eager(mixed):
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth
    wl = synth.config(0)
    prec = hdg.HDG_MIXED if mixed else hdg.HDG_FP64
    print(f"[graph] 4^3 p=2 Newton step, {'mixed' if mixed else 'FP64'}, chunks of 23", flush=True)
    st = pipeline.NewtonStep(wl, prec=prec, chunk=23)
    st.run_calls()
    torch.cuda.synchronize()
    eager = _outputs(st)
    st.run()
    torch.cuda.synchronize()
    one_call = _outputs(st)
    for k in OUTS:
        assert np.array_equal(one_call[k], eager[k]), k
    graph = st.capture()
    other = torch.cuda.Stream()
    x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for rep in range(3):
        y = (x * 2.0).sum()          # unrelated eager work between replays
        torch.cuda.synchronize()
        for k in OUTS:
            getattr(st, k).fill_(float("nan") if getattr(st, k).dtype.is_floating_point else 0)
        graph.replay(other if rep == 1 else None)
        torch.cuda.synchronize()
        got = _outputs(st)
        for k in OUTS:
            assert np.array_equal(got[k], eager[k], equal_nan=False), (rep, k)
        assert np.isfinite(float(y))
    # new input contents: the replay and an eager step on the same inputs agree
    st.U.add_(1e-4 * torch.sin(torch.arange(st.U.numel(), device="cuda", dtype=torch.float64)))
    graph.replay()
    torch.cuda.synchronize()
    got = _outputs(st)
    st.run()
    torch.cuda.synchronize()
    ref = _outputs(st)
    for k in OUTS:
        assert np.array_equal(got[k], ref[k]), k
    assert not np.array_equal(ref["dUhat"], eager["dUhat"])
    graph.close()


def test_graph_capture_rejects_the_default_stream():
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth
    wl = synth.config(0, n_override=2)
    st = pipeline.NewtonStep(wl)
    args = st.ctx.newton_args(st)
    g = hdg._vp()
    import ctypes
    assert st.ctx.L.hdg_graph_capture_newton(st.ctx.h, ctypes.byref(args), ctypes.byref(g), None) == -1
    bad = st.ctx.newton_args(st)
    bad.gmres_m = 0
    assert st.ctx.L.hdg_newton_step(st.ctx.h, ctypes.byref(bad), None) == -1
    bad = st.ctx.newton_args(st)
    bad.cond_work_bytes = 16
    assert st.ctx.L.hdg_newton_step(st.ctx.h, ctypes.byref(bad), None) == -5
    torch.cuda.synchronize()
