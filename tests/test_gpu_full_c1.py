"""Full-mesh parity on the 8^3 p=3 supersonic Taylor-Green workload (512
elements), FP64 path and mixed path (FP32 factorisation, one FP64-residual
refinement, FP32 Schwarz inverses) against the oracle's condensation of every
element:

* every element's S^K and g^K, the assembled S (Frobenius over the blocks) and
  g (2-norm): 1e-12 for FP64, 1e-10 for the mixed path;
* the GMRES(30) increment: on identical S and g (1e-12), and end to end
  against the oracle's own S and g, held to the first-order effect of the S
  and g differences, ||S^{-1} [(g_gpu - g) - (S_gpu - S) x]|| (GMRES(30)
  converges to rounding on this workload, so the increment is the solution
  of S x = g and the bound is that of a perturbed linear system);
* the FP32 Schwarz apply at p = 3 and p = 4 against the oracle's FP64 LU solves
  of the same patch matrices, within f cond(S_r) u_32.
"""
import os

import numpy as np
import pytest

from gpu_common import O, RTOL_FP64, assert_rel, bsr_blocks, rel_err, sk_view

pytestmark = pytest.mark.gpu

RTOL_MIXED = 1e-10


def _oracle_all(wl):
    """S^K, g^K of every element (element systems not kept)."""
    from concurrent.futures import ThreadPoolExecutor
    sz = O.Sizes(wl.mesh)

    def one(e):
        S, g, _ = O.condense(O.element_system(wl, e, sz), sz.n(e))
        return S, g

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, range(wl.mesh.n_elem)))


def _bsr_rel(blocks, ts):
    num = sum(np.linalg.norm(blocks[k] - ts.blocks[k]) ** 2 for k in ts.blocks) ** 0.5
    den = sum(np.linalg.norm(ts.blocks[k]) ** 2 for k in ts.blocks) ** 0.5
    return num / den


@pytest.fixture(scope="module")
def c1all():
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth
    wl = synth.config(1)
    print("[c1 full] FP64 Newton step on cuda:0", flush=True)
    st = pipeline.NewtonStep(wl)
    st.run_calls()
    torch.cuda.synchronize()
    fp64 = dict(SK=st.SK.cpu().numpy(), S=st.S.cpu().numpy(), g=st.g.cpu().numpy(), dUhat=st.dUhat.cpu().numpy(),
                hist=st.hist.cpu().numpy(), info=st.info.cpu().numpy())
    print("[c1 full] mixed Newton step", flush=True)
    stm = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, ctx=st.ctx, share=st)
    stm.run_calls()
    torch.cuda.synchronize()
    mixed = dict(SK=stm.SK.cpu().numpy(), S=stm.S.cpu().numpy(), g=stm.g.cpu().numpy(),
                 dUhat=stm.dUhat.cpu().numpy(), hist=stm.hist.cpu().numpy(), info=stm.info.cpu().numpy())
    print("[c1 full] oracle condensation of all 512 elements", flush=True)
    ora = _oracle_all(wl)
    ts = O.TraceSystem(wl, [o[0] for o in ora], [o[1] for o in ora])
    print("[c1 full] oracle GMRES(30)", flush=True)
    x, hx = O.gmres(ts, ts.g, wl.gmres_m)
    return dict(wl=wl, ctx=st.ctx, fp64=fp64, mixed=mixed, ora=ora, ts=ts, x=x, hx=hx)


@pytest.mark.parametrize("path,tol", [("fp64", RTOL_FP64), ("mixed", RTOL_MIXED)])
def test_every_element_and_the_assembled_system(c1all, path, tol):
    gpu, ora, ts, ctx = c1all[path], c1all["ora"], c1all["ts"], c1all["ctx"]
    assert np.all(gpu["info"] == 0)
    ws = wg = 0.0
    for e in range(len(ora)):
        S, g = sk_view(ctx, gpu["SK"], e)
        ws = max(ws, rel_err(S, ora[e][0]))
        wg = max(wg, rel_err(g, ora[e][1]))
    es = _bsr_rel(bsr_blocks(ctx, gpu["S"]), ts)
    eg = rel_err(gpu["g"], ts.g)
    print(f"  {path}: max over 512 elements S^K {ws:.2e} g^K {wg:.2e}; assembled S {es:.2e} g {eg:.2e}")
    assert ws <= tol and wg <= tol and es <= tol and eg <= tol


def test_fp64_increment_on_identical_inputs(c1all):
    wl, ctx, gpu = c1all["wl"], c1all["ctx"], c1all["fp64"]
    tsg = O.TraceSystem.from_blocks(wl, bsr_blocks(ctx, gpu["S"]), gpu["g"])
    xg, _ = O.gmres(tsg, tsg.g, wl.gmres_m)
    assert_rel(gpu["dUhat"], xg, RTOL_FP64, "dUhat, same S and g")


def _first_order(c1all, gpu):
    """||S^{-1} [(g_gpu - g) - (S_gpu - S) x]|| by the oracle's GMRES on its own S."""
    wl, ctx, ts, x = c1all["wl"], c1all["ctx"], c1all["ts"], c1all["x"]
    tsg = O.TraceSystem.from_blocks(wl, bsr_blocks(ctx, gpu["S"]), gpu["g"])
    d = (gpu["g"] - ts.g) - (tsg.matvec(x) - ts.matvec(x))
    dx, dh = O.gmres(ts, d, wl.gmres_m)
    assert dh[-1] <= 1e-12 * dh[0]
    return np.linalg.norm(dx)


def test_fp64_increment_end_to_end(c1all):
    gpu, x, hx = c1all["fp64"], c1all["x"], c1all["hx"]
    assert hx[-1] <= 1e-12 * hx[0] and gpu["hist"][-1] <= 1e-12 * gpu["hist"][0]  # both converged
    err = np.linalg.norm(gpu["dUhat"] - x)
    pred = _first_order(c1all, gpu)
    nx = np.linalg.norm(x)
    print(f"  FP64 dUhat end to end: {err / nx:.3e}; first-order effect of the S, g differences {pred / nx:.3e}")
    assert err <= 2.0 * pred + RTOL_FP64 * nx


def test_mixed_increment_end_to_end(c1all):
    """The mixed path's increment (FP32 Schwarz inverses, GMRES(30)) against the
    oracle's FP64 increment: converged on both sides, so it differs by the
    first-order effect of the S, g differences and the GMRES stopping level."""
    gpu, x, hx = c1all["mixed"], c1all["x"], c1all["hx"]
    h = gpu["hist"]
    print(f"  mixed GMRES residual reduction {h[-1] / h[0]:.2e}")
    assert h[-1] <= 1e-12 * h[0]
    err = np.linalg.norm(gpu["dUhat"] - x)
    pred = _first_order(c1all, gpu)
    nx = np.linalg.norm(x)
    print(f"  mixed dUhat: {err / nx:.3e} relative to the FP64 oracle; first-order prediction {pred / nx:.3e}")
    assert err <= 2.0 * pred + 1e-11 * nx
    assert err <= RTOL_MIXED * nx


@pytest.mark.parametrize("p,n", [(3, 3), (4, 3)])
def test_fp32_schwarz_apply(p, n):
    """FP32 Schwarz inverses (set-up and apply) at p = 3 and 4 against the
    oracle's FP64 LU solves of the GPU's own patch matrices."""
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth
    mesh = synth.box_mesh((n, n, n), p=p, perturb=0.05, seed=p)
    wl = synth.make_state(mesh, lambda x: synth.tgv_state(x, 1.25), mach=1.25, noise=1e-3, seed=p)
    print(f"[c1 full] FP32 Schwarz blocks, {n}^3 p={p}", flush=True)
    st = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED)
    st.residual_jacobian()
    st.condense()
    st.assemble()
    st.asm_setup()
    torch.cuda.synchronize()
    assert not st.asm_info.any().item()
    ts = O.TraceSystem.from_blocks(wl, bsr_blocks(st.ctx, st.S.cpu().numpy()), st.g.cpu().numpy())
    x = torch.as_tensor(wl.x, dtype=torch.float64, device="cuda")
    z = torch.empty_like(x)
    work = torch.empty(st.ctx.workspace_size(3), dtype=torch.uint8, device="cuda")
    st.ctx.hdg_asm_block_apply(1, st.Sinv, x, z, work)
    torch.cuda.synchronize()
    err = rel_err(z.cpu().numpy(), ts.asm_apply(wl.x))
    f = int(st.ctx.layout["elem_f"][0])
    cond = max(np.linalg.cond(ts.patch_matrix(r)) for r in range(mesh.n_elem))
    bound = f * cond * float(np.finfo(np.float32).eps)
    print(f"  p={p}: M^-1 x (FP32 inverses) {err:.3e}; bound f cond(S_r) u32 = {bound:.3e} (max cond {cond:.1f})")
    assert err <= bound
