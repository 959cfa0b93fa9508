"""GPU parity of the artificial-viscosity field (hdg_av_field: the sensor of
eq. av-coeffs and the smoothing S_h) against the oracle (oracle/av.py), and of
a DIRK step with the lagged viscosity (recomputed at the start of the step,
frozen during it)."""
import math

import numpy as np
import pytest

from gpu_common import O, assert_rel

pytestmark = pytest.mark.gpu

PRM = dict(c_av=2e-3, h_m=2 * math.pi / 3, eps=1e-10, s_max=math.inf, rho_min=1e-8, p_min=1e-8)


def _compressive(n=3, p=2, periodic=(True, True, True), seed=2, noise=0.0):
    from paper_2608_27863_amd import synth
    L = (2 * math.pi, 2 * math.pi if periodic[1] else 1.0, 2 * math.pi)
    mesh = synth.box_mesh((n, n, n), lengths=L, periodic=periodic, p=p, perturb=0.1, seed=seed)

    def field(x):
        u = synth.tgv_state(x, 1.25)
        rho = u[..., 0]
        v1 = u[..., 1] / rho + 0.4 * np.sin(x[..., 0])
        pr = 0.4 * (u[..., 4] - 0.5 * (u[..., 1] ** 2 + u[..., 2] ** 2 + u[..., 3] ** 2) / rho)
        return np.stack(synth._conserved(rho, v1, u[..., 2] / rho, u[..., 3] / rho, pr), axis=-1)

    return synth.make_state(mesh, field, mach=1.25, noise=noise, seed=seed, reynolds=400.0, gmres_m=40,
                            boundary_field=field)


@pytest.mark.parametrize("periodic", [(True, True, True), (True, False, True)])
@pytest.mark.parametrize("iters", [0, 1, 2])
def test_av_field_matches_oracle(periodic, iters):
    import torch
    from oracle import av as AV
    from paper_2608_27863_amd import hdg
    wl = _compressive(periodic=periodic)
    print(f"[av] 3^3 p=2 {'periodic' if all(periodic) else 'walls in y'}, {iters} smoothing passes", flush=True)
    ctx = hdg.Context(wl.mesh, wl)
    f64 = dict(dtype=torch.float64, device="cuda")
    U, Q = torch.as_tensor(wl.U, **f64), torch.as_tensor(wl.Q, **f64)
    nu = torch.full((int(ctx.layout["node_off"][-1]),), float("nan"), **f64)
    raw = torch.empty(ctx.n_elem, **f64)
    work = torch.empty(ctx.workspace_size(7), dtype=torch.uint8, device="cuda")
    ctx.hdg_av_field(dict(PRM, smooth_iters=iters), U, Q, nu, work, nu_raw=raw)
    torch.cuda.synchronize()
    nu_o, raw_o = AV.av_field(wl, wl.U, wl.Q, PRM, iters)
    assert raw_o.max() > 1e-6
    assert_rel(raw.cpu().numpy(), raw_o, 1e-13, "raw elemental viscosity")
    assert_rel(nu.cpu().numpy(), nu_o, 1e-13, "nodal viscosity")


def test_dirk_step_with_lagged_viscosity():
    import torch
    from oracle import av as AV
    from oracle import newton as N
    from paper_2608_27863_amd import pipeline
    wl = _compressive(n=2, p=1, noise=1e-3, seed=5)
    prm = dict(PRM, h_m=math.pi, c_av=5e-2, smooth_iters=2)
    print("[av] DIRK step with lagged artificial viscosity, 2^3 p=1", flush=True)
    st = pipeline.NewtonStep(wl, m=wl.gmres_m)
    stepper = pipeline.DirkStepper(pipeline.NewtonSolver(st, tol=1e-11, maxit=8), av=prm)
    hists = stepper.step()
    torch.cuda.synchronize()
    nu_o, _ = AV.av_field(wl, wl.U, wl.Q, PRM | dict(h_m=math.pi, c_av=5e-2), 2)
    assert nu_o.max() > 1e-5
    wl.nu = nu_o
    Qo, Uo, Uho, ho = N.dirk_step(wl, wl.Q, wl.U, wl.Uhat, m=wl.gmres_m, tol=1e-11, maxit=8)
    assert [len(h) for h in hists] == [len(h) for h in ho]
    assert_rel(st.nu.cpu().numpy(), nu_o, 1e-13, "lagged viscosity")
    for name, got, ref in (("Q", st.Q, Qo), ("U^{n+1}", st.U, Uo), ("Uhat", st.Uhat, Uho)):
        assert_rel(got.cpu().numpy(), ref, 1e-11, name)
