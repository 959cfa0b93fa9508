"""hdg_asm_block_apply_noalloc (library-owned scratch, no allocation) against
hdg_asm_block_apply (caller workspace) through the C ABI: the same kernels in
the same order, so the results must be bit-identical.  Two calls in a row on
one GPU, the second on a smaller mesh (the shared array keeps the first
call's contents), for FP64 and FP32 Schwarz inverses; a mesh needing more
than the array is rejected before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _schwarz(wl, prec):
    import torch
    from paper_2608_27863_amd import pipeline
    st = pipeline.NewtonStep(wl, asm_prec=prec)
    st.residual_jacobian()
    st.condense()
    st.assemble()
    st.asm_setup()
    torch.cuda.synchronize()
    assert not st.asm_info.any().item()
    return st


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_apply_matches_workspace_apply(prec):
    import torch
    from paper_2608_27863_amd import synth
    cases = [synth.config(0), synth.config(0, n_override=2)]
    cases[1].mesh.elem_p[:] = 1  # a smaller second call (p = 1)
    cases[1] = synth.make_state(cases[1].mesh, lambda x: synth.tgv_state(x, 0.1), mach=0.1, noise=1e-3, seed=2)
    for k, wl in enumerate(cases):
        print(f"[noalloc] call {k}: {wl.mesh.n_elem} elements, p={int(wl.mesh.elem_p[0])}, prec={prec}", flush=True)
        st = _schwarz(wl, prec)
        ctx = st.ctx
        r = torch.as_tensor(np.random.default_rng(k).standard_normal(ctx.N_uh), device="cuda")
        z_ref = torch.empty_like(r)
        z_new = torch.full_like(r, float("nan"))
        work = torch.empty(ctx.workspace_size(3, prec), dtype=torch.uint8, device="cuda")
        ctx.hdg_asm_block_apply(prec, st.Sinv, r, z_ref, work)
        ctx.hdg_asm_block_apply_noalloc(prec, st.Sinv, r, z_new)
        torch.cuda.synchronize()
        a, b = z_ref.cpu().numpy(), z_new.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b), np.abs(a - b).max()


def test_noalloc_apply_rejects_a_mesh_beyond_the_array():
    import torch
    from paper_2608_27863_amd import hdg, synth
    mesh = synth.box_mesh((18, 18, 18), p=4)  # 5832 elements x 750 trace values > 4194304
    wl = synth.Workload("big", mesh, 1.25, 1600.0, 1.4, 0.71, 5.0, 0.01, synth.dirk_alpha(), 1,
                        *([np.zeros(1)] * 7), 1, 0)
    ctx = hdg.Context(mesh, wl)
    assert int(ctx.layout["elem_f"].sum()) > 4194304
    d = torch.zeros(16, dtype=torch.float64, device="cuda")
    rc = ctx.L.hdg_asm_block_apply_noalloc(ctx.h, 0, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(d.data_ptr()),
                                           ctypes.c_void_p(d[8:].data_ptr()), None)
    assert rc == -5
    ctx.close()
