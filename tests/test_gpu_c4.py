"""The 12^3 periodic supersonic Taylor-Green mesh at p = 4 (1728 elements,
n = 2500, f = 750): the largest single-GPU partition.  Condensation streams in
chunks of 256 elements, GMRES(50) uses FP32 Schwarz inverses, and the whole
step is replayed from a HIP graph.  Sampled elements against the oracle; GMRES
and recovery checked through properties that hold at any size."""
import numpy as np
import pytest

from gpu_common import O, RTOL_FP64, oracle_condensed, recovery_checks, rel_err, sk_view

pytestmark = pytest.mark.gpu

SAMPLE = (0, 1727)


@pytest.fixture(scope="module")
def c4():
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth
    wl = synth.config(4)
    print("[c4] 12^3 p=4: FP64 step, chunks of 256, FP32 Schwarz, GMRES(50), captured in a graph", flush=True)
    st = pipeline.NewtonStep(wl, prec=hdg.HDG_FP64, asm_prec=hdg.HDG_MIXED, chunk=256)
    graph = st.capture()
    graph.replay()
    torch.cuda.synchronize()
    gpu = dict(SK=st.SK.cpu().numpy(), dUhat=st.dUhat.cpu().numpy(), hist=st.hist.cpu().numpy(),
               info=st.info.cpu().numpy(), asm_info=st.asm_info.cpu().numpy())
    no = st.ctx.layout["node_off"]
    gpu["dQU"] = {e: st.dQU[20 * int(no[e]):20 * int(no[e + 1])].cpu().numpy() for e in SAMPLE}
    print("[c4] FP64 step done; oracle on sampled elements", flush=True)
    ora = oracle_condensed(wl, SAMPLE, threads=len(SAMPLE))
    return dict(wl=wl, st=st, gpu=gpu, ora=ora)


def test_c4_sampled_condensation(c4):
    gpu, ora, st = c4["gpu"], c4["ora"], c4["st"]
    assert np.all(gpu["info"] == 0)
    for e in SAMPLE:
        S, g = sk_view(st.ctx, gpu["SK"], e)
        es, eg = rel_err(S, ora[e]["SK"]), rel_err(g, ora[e]["gK"])
        print(f"  element {e}: S^K {es:.2e}  g^K {eg:.2e}")
        assert es <= RTOL_FP64 and eg <= RTOL_FP64


def test_c4_gmres_fp32_schwarz(c4):
    h = c4["gpu"]["hist"]
    assert np.all(c4["gpu"]["asm_info"] == 0)
    assert h.shape == (51,)
    print(f"  preconditioned residual: {h[0]:.3e} -> {h[-1]:.3e} in 50 iterations")
    assert np.all(np.diff(h) <= 1e-14 * h[0]) and h[-1] < 1e-6 * h[0]


def test_c4_sampled_recovery(c4):
    wl, gpu, ora = c4["wl"], c4["gpu"], c4["ora"]
    for e in SAMPLE:
        b, fr = recovery_checks(wl, e, ora[e]["E"], ora[e]["X"], gpu["dUhat"], gpu["dQU"][e])
        print(f"  d(Q,U) element {e}: backward {b:.2f} of n u, forward {fr:.2f} of bound")
        assert b <= 1.0 and fr <= 1.0


def test_c4_mixed_condensation(c4):
    """Mixed condensation of the same mesh in chunks of 256, sharing the FP64
    step's buffers."""
    import torch
    from paper_2608_27863_amd import hdg, pipeline
    wl, ora = c4["wl"], c4["ora"]
    print("[c4] mixed condensation", flush=True)
    stm = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, chunk=256, ctx=c4["st"].ctx, share=c4["st"])
    stm.residual_jacobian()
    stm.condense()
    torch.cuda.synchronize()
    assert np.all(stm.info.cpu().numpy() == 0)
    SK = stm.SK.cpu().numpy()
    for e in SAMPLE:
        S, g = sk_view(stm.ctx, SK, e)
        es, eg = rel_err(S, ora[e]["SK"]), rel_err(g, ora[e]["gK"])
        print(f"  element {e}: S^K {es:.2e}  g^K {eg:.2e}")
        assert es <= 1e-10 and eg <= 1e-10
