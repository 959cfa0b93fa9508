"""A whole Newton step captured in a HIP graph (torch.cuda.CUDAGraph): every
replay must reproduce the eager step bit for bit, with the program's own eager
work and synchronisations between replays, and must follow new contents of
the input buffers."""
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
    st.run()
    torch.cuda.synchronize()
    eager = _outputs(st)
    graph = st.capture()
    x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for rep in range(3):
        y = (x * 2.0).sum()          # unrelated eager work between replays
        torch.cuda.synchronize()
        for k in OUTS:
            getattr(st, k).fill_(float("nan") if getattr(st, k).dtype.is_floating_point else 0)
        graph.replay()
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
