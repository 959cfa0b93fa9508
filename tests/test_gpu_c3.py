"""The wall-bounded batching workload: 2000 hexahedra (20 x 10 x 10) stretched
toward both walls (ratio 1.15, first-cell aspect ratio 50), 2% trilinear
perturbation, periodic in x and z with Dirichlet-state walls, degrees drawn
from {2, 3, 4}: elements of every size condensed in the same launches.  One
element of each degree, including wall elements, against the oracle."""
import numpy as np
import pytest

from gpu_common import O, RTOL_FP64, oracle_condensed, recovery_checks, rel_err, sk_view

pytestmark = pytest.mark.gpu


def _sample(wl):
    """First wall element and first interior element of each degree."""
    ep = wl.mesh.elem_p
    walls = set()
    for F in np.nonzero(wl.mesh.face_bc)[0]:
        walls.add(int(wl.mesh.face_elem[F][0][0]))
    out = []
    for p in (2, 3, 4):
        es = [e for e in range(wl.mesh.n_elem) if ep[e] == p]
        out.append(next(e for e in es if e in walls))
        out.append(next(e for e in es if e not in walls))
    return sorted(set(out))


@pytest.fixture(scope="module")
def c3():
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth
    wl = synth.config(3)
    sample = _sample(wl)
    counts = {p: int(np.sum(wl.mesh.elem_p == p)) for p in (2, 3, 4)}
    print(f"[c3] {wl.mesh.n_elem} elements, degrees {counts}, walls {int(wl.mesh.face_bc.sum())} faces; "
          f"sample {sample}", flush=True)
    st = pipeline.NewtonStep(wl, prec=hdg.HDG_FP64)
    st.run()
    torch.cuda.synchronize()
    gpu = dict(SK=st.SK.cpu().numpy(), dUhat=st.dUhat.cpu().numpy(), hist=st.hist.cpu().numpy(),
               info=st.info.cpu().numpy(), asm_info=st.asm_info.cpu().numpy())
    no = st.ctx.layout["node_off"]
    gpu["dQU"] = {e: st.dQU[20 * int(no[e]):20 * int(no[e + 1])].cpu().numpy() for e in sample}
    print("[c3] FP64 step done; oracle on sampled elements", flush=True)
    ora = oracle_condensed(wl, sample, threads=len(sample))
    return dict(wl=wl, st=st, gpu=gpu, ora=ora, sample=sample)


def test_c3_sampled_condensation(c3):
    gpu, ora, st, wl = c3["gpu"], c3["ora"], c3["st"], c3["wl"]
    assert np.all(gpu["info"] == 0)
    for e in c3["sample"]:
        S, g = sk_view(st.ctx, gpu["SK"], e)
        es, eg = rel_err(S, ora[e]["SK"]), rel_err(g, ora[e]["gK"])
        print(f"  element {e} (p={int(wl.mesh.elem_p[e])}): S^K {es:.2e}  g^K {eg:.2e}")
        assert es <= RTOL_FP64 and eg <= RTOL_FP64


def test_c3_gmres_and_recovery(c3):
    wl, gpu, ora = c3["wl"], c3["gpu"], c3["ora"]
    h = gpu["hist"]
    assert np.all(gpu["asm_info"] == 0)
    print(f"  preconditioned residual {h[0]:.3e} -> {h[-1]:.3e} in {len(h) - 1} iterations")
    assert np.all(np.diff(h) <= 1e-13 * h[0]) and h[-1] < h[0]
    for e in c3["sample"]:
        b, fr = recovery_checks(wl, e, ora[e]["E"], ora[e]["X"], gpu["dUhat"], gpu["dQU"][e])
        assert b <= 1.0 and fr <= 1.0, (e, b, fr)


def test_c3_mixed_condensation(c3):
    import torch
    from paper_2608_27863_amd import hdg, pipeline
    wl, ora = c3["wl"], c3["ora"]
    print("[c3] mixed condensation", flush=True)
    stm = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, ctx=c3["st"].ctx, share=c3["st"])
    stm.residual_jacobian()
    stm.condense()
    torch.cuda.synchronize()
    assert np.all(stm.info.cpu().numpy() == 0)
    SK = stm.SK.cpu().numpy()
    for e in c3["sample"]:
        S, g = sk_view(stm.ctx, SK, e)
        es, eg = rel_err(S, ora[e]["SK"]), rel_err(g, ora[e]["gK"])
        print(f"  element {e} (p={int(wl.mesh.elem_p[e])}): S^K {es:.2e}  g^K {eg:.2e}")
        assert es <= 1e-10 and eg <= 1e-10
