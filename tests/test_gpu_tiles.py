"""The two tile shapes of the trailing update (128 x 128 and 256 x 128) give
bit-identical condensations and Schwarz inverses (each output's products are
accumulated in the same order), for FP64 and mixed precision, degrees 1-4,
mixed-degree ragged chunks; and the autotuner picks one of them per size of
system and leaves the results unchanged."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _wl_mixed_degrees():
    from paper_2608_27863_amd import synth
    rng = np.random.default_rng(3)
    pe = rng.choice([1, 2, 3, 4], size=3 * 3 * 2)
    mesh = synth.group_by_degree(synth.box_mesh((3, 3, 2), p=pe, perturb=0.05, seed=3))
    return synth.make_state(mesh, lambda x: synth.tgv_state(x, 1.25), mach=1.25, noise=1e-3, nu_amp=3e-4, seed=3,
                            gmres_m=12)


def _outputs(st):
    return {k: getattr(st, k).cpu().numpy().copy() for k in ("E", "SK", "S", "g", "Sinv", "dUhat", "dQU")}


@pytest.mark.parametrize("prec", [0, 1])
def test_tile_shapes_are_bit_identical(prec):
    import torch
    from paper_2608_27863_amd import pipeline
    wl = _wl_mixed_degrees()
    print(f"[tiles] degrees 1-4, ragged chunks of 5, prec {prec}", flush=True)
    st = pipeline.NewtonStep(wl, prec=prec, chunk=5)
    ref = None
    for rows in (128, 256):
        st.ctx.hdg_set_update_tile(0, rows)
        assert st.ctx.hdg_get_update_tile(2500) == rows
        st.run_calls()
        torch.cuda.synchronize()
        assert not st.info.any().item() and not st.asm_info.any().item()
        out = _outputs(st)
        if ref is None:
            ref = out
        else:
            for k in out:
                assert np.array_equal(out[k], ref[k]), k


def test_autotuner_keeps_results():
    import torch
    from paper_2608_27863_amd import pipeline, synth
    wl = synth.config(0)
    st = pipeline.NewtonStep(wl)
    st.run_calls()
    torch.cuda.synchronize()
    ref = _outputs(st)
    table = pipeline.autotune_update_tiles(st, log=print)
    assert set(table) == {540, 272} and all(v[0] in (128, 256) for v in table.values())
    st.run_calls()
    torch.cuda.synchronize()
    out = _outputs(st)
    for k in ("SK", "S", "g", "Sinv", "dUhat", "dQU"):
        assert np.array_equal(out[k], ref[k]), k
