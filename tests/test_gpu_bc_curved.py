"""GPU parity of the boundary types (prescribed state, extrapolated state,
isothermal and adiabatic no-slip walls, symmetry; eq. hdg-trace with the weak
boundary statements of section 2.1) and of curved (triquadratic) elements
against the oracle: element systems entry by entry, condensed element
systems, and a whole Newton step."""
import numpy as np
import pytest

from gpu_common import O, RTOL_FP64, assert_rel, bsr_blocks, e_view, rel_err, residual_scale, sk_view

pytestmark = pytest.mark.gpu

ALL_TYPES = {(0, 0): 1, (0, 1): 2, (1, 0): 3, (1, 1): 4, (2, 0): 5, (2, 1): 5}


def _walls_wl(p):
    from paper_2608_27863_amd import synth
    mesh = synth.box_mesh((2, 2, 2), lengths=(2.0, 1.5, 1.0), periodic=(False, False, False), p=p, perturb=0.1,
                          seed=4)
    mesh = synth.set_boundary_types(mesh, ALL_TYPES)
    f = lambda x: synth.tgv_state(x, 0.8)
    return synth.make_state(mesh, f, mach=0.8, noise=1e-2, nu_amp=3e-4, seed=4, reynolds=80.0,
                            boundary_field=f, gmres_m=40)


def _curved_wl(p):
    from paper_2608_27863_amd import synth
    mesh = synth.curve_mesh(synth.box_mesh((2, 2, 2), p=p), 0.2)
    return synth.make_state(mesh, lambda x: synth.tgv_state(x, 1.25), mach=1.25, noise=1e-3, nu_amp=5e-4, seed=3,
                            gmres_m=40)


CASES = {"every boundary type, p=2": lambda: _walls_wl(2), "every boundary type, p=3": lambda: _walls_wl(3),
         "curved, p=2": lambda: _curved_wl(2), "curved, p=4": lambda: _curved_wl(4)}


@pytest.mark.parametrize("case", list(CASES))
def test_element_systems_condensation_and_step(case):
    import torch
    from paper_2608_27863_amd import pipeline
    wl = CASES[case]()
    print(f"[bc/curved] {case}", flush=True)
    st = pipeline.NewtonStep(wl, m=wl.gmres_m)
    st.residual_jacobian()
    torch.cuda.synchronize()
    E = st.E.cpu().numpy()
    st.condense()
    st.assemble()
    st.asm_setup()
    st.gmres()
    st.recover()
    torch.cuda.synchronize()
    ctx = st.ctx
    sz = O.Sizes(wl.mesh)
    SK = st.SK.cpu().numpy()
    worst = {}
    for e in range(wl.mesh.n_elem):
        Eg, _ = e_view(ctx, E, e)
        Eo = np.array(O.element_system(wl, e, sz))
        n = sz.n(e)
        for name, gb, ob in zip("A B C D".split(), O.split(Eg, n)[:4], O.split(Eo, n)[:4]):
            worst[name] = max(worst.get(name, 0.0), rel_err(gb, ob))
        scale = residual_scale(wl, ctx, e, Eo)
        worst["R"] = max(worst.get("R", 0.0), np.linalg.norm(Eg[:, -1] - Eo[:, -1]) / np.linalg.norm(scale))
        So, go, _ = O.condense(Eo, n)
        S, g = sk_view(ctx, SK, e)
        worst["S^K"] = max(worst.get("S^K", 0.0), rel_err(S, So))
        worst["g^K"] = max(worst.get("g^K", 0.0), rel_err(g, go))
    print("  worst:", {k: f"{v:.2e}" for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= RTOL_FP64, (k, v)
    assert not st.info.any().item() and not st.asm_info.any().item()
    ts = O.TraceSystem.from_blocks(wl, bsr_blocks(ctx, st.S.cpu().numpy()), st.g.cpu().numpy())
    x, _ = O.gmres(ts, ts.g, wl.gmres_m)
    assert_rel(st.dUhat.cpu().numpy(), x, RTOL_FP64, "dUhat, same S and g")
