"""GPU parity across degrees and mesh shapes, each against the oracle:
p = 1..4 on perturbed (non-affine) periodic meshes, mixed degrees with
Dirichlet walls (block sizes differ per face), ragged chunks, an element that
meets the same face twice, and argument errors."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from gpu_common import (O, RTOL_FP64, assert_rel, bsr_blocks, e_view, oracle_condensed, recovery_checks, rel_err,
                        residual_scale, sk_view)

pytestmark = pytest.mark.gpu


def _wl_periodic(n, p, perturb=0.1, seed=11, m=8):
    from paper_2608_27863_amd import synth
    mesh = synth.box_mesh(n, p=p, perturb=perturb, seed=seed)
    return synth.make_state(mesh, lambda x: synth.tgv_state(x, 1.25), mach=1.25, noise=1e-3, nu_amp=5e-4,
                            seed=seed, gmres_m=m)


def _wl_walls(seed=13):
    from paper_2608_27863_amd import synth
    nx, ny, nz = 3, 3, 2
    yc = np.concatenate([[0.0], np.cumsum(0.05 * 1.15 ** np.arange(ny))])
    rng = np.random.default_rng(seed)
    pe = rng.choice([1, 2, 3], size=nx * ny * nz)
    mesh = synth.box_mesh((nx, ny, nz), lengths=(2.0, float(yc[-1]), 1.0), periodic=(True, False, True),
                          y_coords=yc, perturb=0.05, p=pe, seed=seed)
    f = lambda x: synth.bl_state(x, 0.5, float(yc[-1]))
    return synth.make_state(mesh, f, mach=0.5, noise=1e-3, seed=seed, gmres_m=8, boundary_field=f)


def _run_and_compare(wl, chunk=None, check_gmres=True):
    import torch
    from paper_2608_27863_amd import pipeline
    st = pipeline.NewtonStep(wl, chunk=chunk)
    st.residual_jacobian()
    torch.cuda.synchronize()
    E = st.E.cpu().numpy()
    st.condense()
    st.assemble()
    torch.cuda.synchronize()
    ora = oracle_condensed(wl)
    ctx = st.ctx
    for e in range(wl.mesh.n_elem):
        Eg, _ = e_view(ctx, E, e)
        Eo = ora[e]["E"]
        n = int(ctx.layout["elem_n"][e])
        for name, gb, ob in zip("A B C D".split(), O.split(Eg, n)[:4], O.split(Eo, n)[:4]):
            assert rel_err(gb, ob) <= RTOL_FP64, (e, name, rel_err(gb, ob))
        scale = residual_scale(wl, ctx, e, Eo)
        assert np.linalg.norm(Eg[:, -1] - Eo[:, -1]) <= RTOL_FP64 * np.linalg.norm(scale), e
    assert np.all(st.info.cpu().numpy() == 0)
    SK = st.SK.cpu().numpy()
    for e in range(wl.mesh.n_elem):
        S, g = sk_view(ctx, SK, e)
        assert rel_err(S, ora[e]["SK"]) <= RTOL_FP64 and rel_err(g, ora[e]["gK"]) <= RTOL_FP64, e
    ts = O.TraceSystem(wl, [ora[e]["SK"] for e in range(wl.mesh.n_elem)],
                       [ora[e]["gK"] for e in range(wl.mesh.n_elem)])
    blocks = bsr_blocks(ctx, st.S.cpu().numpy())
    assert set(blocks) == set(ts.blocks)
    num = sum(np.linalg.norm(blocks[k] - ts.blocks[k]) ** 2 for k in blocks) ** 0.5
    den = sum(np.linalg.norm(ts.blocks[k]) ** 2 for k in blocks) ** 0.5
    assert num / den <= RTOL_FP64
    if check_gmres:
        st.asm_setup()
        st.gmres()
        st.recover()
        torch.cuda.synchronize()
        assert np.all(st.asm_info.cpu().numpy() == 0)
        tsg = O.TraceSystem.from_blocks(wl, blocks, st.g.cpu().numpy())
        x, hist = O.gmres(tsg, tsg.g, wl.gmres_m)
        assert_rel(st.dUhat.cpu().numpy(), x, RTOL_FP64, "dUhat (same S, g)")
        dQU = st.dQU.cpu().numpy()
        sz = O.Sizes(wl.mesh)
        no = ctx.layout["node_off"]
        for e in range(wl.mesh.n_elem):
            b, fr = recovery_checks(wl, e, ora[e]["E"], ora[e]["X"], st.dUhat.cpu().numpy(),
                                    dQU[20 * int(no[e]):20 * int(no[e + 1])])
            assert b <= 1.0 and fr <= 1.0, (e, b, fr)
    return st


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_degrees_on_perturbed_periodic_mesh(p):
    print(f"[shapes] p={p}, 2x2x2 perturbed periodic", flush=True)
    _run_and_compare(_wl_periodic((2, 2, 2), p))


def test_mixed_degrees_dirichlet_walls_ragged_chunks():
    print("[shapes] mixed p, Dirichlet walls, chunks of 5", flush=True)
    wl = _wl_walls()
    assert wl.mesh.face_bc.sum() > 0 and len(set(wl.mesh.elem_p.tolist())) > 1
    _run_and_compare(wl, chunk=5)


def _mixed_condense_and_compare(wl, chunk=None):
    """Mixed condensation against the oracle: S^K and g^K to 1e-10 relative per
    element; the stored X = A^{-1}[B | R_qu] within 10x of the same recipe run
    through LAPACK (FP32 LU, one FP64-residual refinement step)."""
    import torch
    from paper_2608_27863_amd import hdg, pipeline
    st = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, chunk=chunk)
    st.residual_jacobian()
    st.condense()
    torch.cuda.synchronize()
    assert np.all(st.info.cpu().numpy() == 0)
    ora = oracle_condensed(wl)
    ctx = st.ctx
    SK, E = st.SK.cpu().numpy(), st.E.cpu().numpy()
    worst = [0.0, 0.0, 0.0]
    ref = 0.0
    for e in range(wl.mesh.n_elem):
        S, g = sk_view(ctx, SK, e)
        n, f = int(ctx.layout["elem_n"][e]), int(ctx.layout["elem_f"][e])
        o = ctx.layout["E_off"]
        a = E[int(o[e]):int(o[e + 1])]
        X = a.reshape(n + f, a.size // (n + f))[:n, n:n + f + 1]
        errs = (rel_err(S, ora[e]["SK"]), rel_err(g, ora[e]["gK"]), rel_err(X, ora[e]["X"]))
        worst = [max(w, x) for w, x in zip(worst, errs)]
        Eo = ora[e]["E"]
        lu = sla.lu_factor(Eo[:n, :n].astype(np.float32))
        solve = lambda R: sla.lu_solve(lu, R.astype(np.float32)).astype(np.float64)
        X0 = solve(Eo[:n, n:])
        ref = max(ref, rel_err(X0 + solve(Eo[:n, n:] - Eo[:n, :n] @ X0), ora[e]["X"]))
    print(f"  mixed: S^K {worst[0]:.2e}  g^K {worst[1]:.2e}  X {worst[2]:.2e} (LAPACK recipe {ref:.2e})", flush=True)
    assert worst[0] <= 1e-10 and worst[1] <= 1e-10 and worst[2] <= max(10.0 * ref, 1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mixed_precision_degrees(p):
    print(f"[shapes] mixed precision, p={p}, 2x2x2 perturbed periodic", flush=True)
    _mixed_condense_and_compare(_wl_periodic((2, 2, 2), p))


def test_mixed_precision_mixed_degrees_ragged_chunks():
    print("[shapes] mixed precision, mixed p, Dirichlet walls, chunks of 5", flush=True)
    _mixed_condense_and_compare(_wl_walls(), chunk=5)


def test_element_meeting_a_face_twice():
    """1 x 2 x 2 periodic: each element's -x and +x faces are the same face.
    Residual, condensation and assembly are defined; the Schwarz patch is
    not (its restriction repeats unknowns), so set-up reports unsupported."""
    import torch
    from paper_2608_27863_amd import hdg
    print("[shapes] 1x2x2 periodic", flush=True)
    wl = _wl_periodic((1, 2, 2), 2, perturb=0.0)
    st = _run_and_compare(wl, check_gmres=False)
    with pytest.raises(hdg.HDGError, match="unsupported"):
        st.asm_setup()


def test_argument_errors_reach_no_kernel():
    import torch
    from paper_2608_27863_amd import hdg, pipeline
    wl = _wl_periodic((2, 2, 2), 1)
    st = pipeline.NewtonStep(wl)
    with pytest.raises(hdg.HDGError, match="invalid argument"):
        st.ctx.hdg_condense(0, 1, 0, 0, st.E, st.SK, st.info, st.cond_work)      # empty chunk
    with pytest.raises(hdg.HDGError, match="invalid argument"):
        st.ctx.hdg_condense(0, 1, 5, 4, st.E, st.SK, st.info, st.cond_work)      # past the end
    with pytest.raises(hdg.HDGError, match="workspace"):
        st.ctx.hdg_condense(0, 1, 0, 8, st.E, st.SK, st.info, st.cond_work[:16])
    with pytest.raises(hdg.HDGError):
        st.ctx.hdg_face_matvec(st.S, st.g, st.g)                                 # aliasing
    with pytest.raises(hdg.HDGError, match="invalid argument"):
        st.ctx.hdg_gmres(0, st.S, st.Sinv, st.g, 0, st.dUhat, st.hist, st.gm_work)  # m = 0


def test_bsr_pattern_on_device():
    """hdg_bsr_pattern hands out the context's device copy of the pattern of S:
    equal to the host layout, and row F holds exactly the faces that share an
    element with F (eq. schur-trace), ascending."""
    import ctypes
    from paper_2608_27863_amd import hdg
    wl = _wl_walls()
    mesh = wl.mesh
    ctx = hdg.Context(mesh, wl)
    try:
        nnzb, rp_dev, col_dev = ctx.hdg_bsr_pattern()
        print(f"[bsr] {mesh.n_face} faces, {nnzb} blocks", flush=True)
        assert nnzb == len(ctx.layout["bsr_col"]) and rp_dev and col_dev
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        rp = np.zeros(mesh.n_face + 1, dtype=np.int32)
        col = np.zeros(nnzb, dtype=np.int32)
        assert hip.hipMemcpy(rp.ctypes.data, rp_dev, rp.nbytes, 2) == 0  # device to host
        assert hip.hipMemcpy(col.ctypes.data, col_dev, col.nbytes, 2) == 0
        assert np.array_equal(rp, ctx.layout["bsr_row_ptr"]) and np.array_equal(col, ctx.layout["bsr_col"])
        for F in range(mesh.n_face):
            elems = {int(mesh.face_elem[F, s, 0]) for s in range(2) if mesh.face_elem[F, s, 0] >= 0}
            want = sorted({int(G) for e in elems for G in mesh.elem_face[e]})
            assert list(col[rp[F]:rp[F + 1]]) == want, F
        only = ctypes.c_int(-7)
        assert ctx.L.hdg_bsr_pattern(ctx.h, ctypes.byref(only), None, None) == 0 and only.value == nnzb
    finally:
        ctx.close()


@pytest.mark.parametrize("case", ["p1", "p3", "p4", "walls"])
def test_matvec_and_schwarz_apply_on_every_block_shape(case):
    """The face matvec (blocks on 128-byte lines streamed through LDS) and the
    FP64 Schwarz apply (streamed or per-row-band, by column alignment) against
    the oracle's products with the GPU's own assembled blocks: block sides
    20 (p=1), 80 (p=3), 125 (p=4, columns off the line boundary) and mixed
    sides on the walled mesh."""
    import torch
    from paper_2608_27863_amd import pipeline
    wl = _wl_walls() if case == "walls" else _wl_periodic((2, 2, 2), int(case[1:]))
    print(f"[shapes] matvec and Schwarz apply, {case}", flush=True)
    st = pipeline.NewtonStep(wl)
    st.residual_jacobian()
    st.condense()
    st.assemble()
    st.asm_setup()
    torch.cuda.synchronize()
    assert not st.info.any().item() and not st.asm_info.any().item()
    ctx = st.ctx
    ts = O.TraceSystem.from_blocks(wl, bsr_blocks(ctx, st.S.cpu().numpy()), st.g.cpu().numpy())
    x = torch.as_tensor(wl.x, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    ctx.hdg_face_matvec(st.S, x, y)
    z = torch.empty_like(x)
    work = torch.empty(ctx.workspace_size(3), dtype=torch.uint8, device="cuda")
    ctx.hdg_asm_block_apply(0, st.Sinv, x, z, work)
    torch.cuda.synchronize()
    assert_rel(y.cpu().numpy(), ts.matvec(wl.x), RTOL_FP64, "S x")
    assert_rel(z.cpu().numpy(), ts.asm_apply(wl.x), RTOL_FP64, "M^-1 x")
    # the padding after every block of S and of the Schwarz inverses is zero
    vo, ao = ctx.layout["bsr_val_off"], ctx.layout["asm_off"]
    assert all(int(o) % 16 == 0 for o in vo) and all(int(o) % 32 == 0 for o in ao)
    Sh, Ih = st.S.cpu().numpy(), st.Sinv.cpu().numpy()
    rp, fo, fs = ctx.layout["bsr_row_ptr"], ctx.layout["face_off"], ctx.layout["elem_f"]
    for F in range(ctx.n_face):
        for k in range(int(rp[F]), int(rp[F + 1])):
            G = int(ctx.layout["bsr_col"][k])
            end = int(vo[k]) + int(fo[F + 1] - fo[F]) * int(fo[G + 1] - fo[G])
            assert not Sh[end:int(vo[k + 1])].any(), (F, G)
    for e in range(ctx.n_elem):
        assert not Ih[int(ao[e]) + int(fs[e]) ** 2:int(ao[e + 1])].any(), e
