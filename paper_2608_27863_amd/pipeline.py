"""One Newton step of the HDG hot path on the GPU, as a sequence of libhdg calls.

Allocates the device buffers (torch) and issues, on one stream:
  hdg_local_residual_jacobian (per chunk) -> hdg_condense (per chunk)
  -> hdg_assemble_trace -> hdg_asm_setup -> hdg_gmres -> hdg_recover_interior.
No arithmetic happens here; every step runs in libhdg's kernels.
"""
from __future__ import annotations

import numpy as np

from .hdg import HDG_FP64, HDG_MIXED, Context


class NewtonStep:
    def __init__(self, wl, prec=HDG_FP64, refine_steps=1, asm_prec=None, chunk=None, m=None,
                 ctx=None, device="cuda"):
        import torch
        self.wl = wl
        self.prec = prec
        self.refine = refine_steps
        self.asm_prec = prec if asm_prec is None else asm_prec
        self.m = wl.gmres_m if m is None else m
        self.ctx = ctx or Context(wl.mesh, wl)
        c = self.ctx
        ne = c.n_elem
        self.chunk = ne if chunk is None else int(chunk)
        self.chunks = [(e0, min(self.chunk, ne - e0)) for e0 in range(0, ne, self.chunk)]
        f64 = dict(dtype=torch.float64, device=device)
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), **f64)
        self.Q, self.U, self.Un = t(wl.Q), t(wl.U), t(wl.Un)
        self.Uhat, self.nu, self.Ub = t(wl.Uhat), t(wl.nu), t(wl.Ub)
        self.E = torch.empty(int(c.layout["E_off"][-1]), **f64)
        qp = max(c.workspace_size(0, HDG_FP64, e0, n) for e0, n in self.chunks)
        self.qp_work = torch.empty(qp, dtype=torch.uint8, device=device)
        cw = max(c.workspace_size(1, prec, e0, n) for e0, n in self.chunks)
        self.cond_work = torch.empty(cw, dtype=torch.uint8, device=device)
        self.SK = torch.empty(int(c.layout["SK_off"][-1]), **f64)
        self.info = torch.zeros(ne, dtype=torch.int32, device=device)
        self.S = torch.empty(int(c.layout["bsr_val_off"][-1]), **f64)
        self.g = torch.empty(c.N_uh, **f64)
        sdt = torch.float64 if self.asm_prec == HDG_FP64 else torch.float32
        self.Sinv = torch.empty(int(c.layout["asm_off"][-1]), dtype=sdt, device=device)
        self.asm_info = torch.zeros(ne, dtype=torch.int32, device=device)
        self.asm_work = torch.empty(c.workspace_size(2, self.asm_prec), dtype=torch.uint8, device=device)
        self.gm_work = torch.empty(c.workspace_size(4, self.asm_prec, 0, self.m), dtype=torch.uint8, device=device)
        self.dUhat = torch.empty(c.N_uh, **f64)
        self.hist = torch.empty(self.m + 1, **f64)
        self.dQU = torch.empty(20 * int(c.layout["node_off"][-1]), **f64)

    def E_chunk(self, e0, n):
        o = self.ctx.layout["E_off"]
        return self.E[int(o[e0]):int(o[e0 + n])]

    # the steps of the hot path
    def residual_jacobian(self, stream=None):
        for e0, n in self.chunks:
            self.ctx.hdg_local_residual_jacobian(e0, n, self.Q, self.U, self.Un, self.Uhat, self.nu,
                                                 self.Ub if self.wl.mesh.face_bc.any() else None,
                                                 self.E_chunk(e0, n), self.qp_work, stream)

    def condense(self, stream=None):
        for e0, n in self.chunks:
            self.ctx.hdg_condense(self.prec, self.refine, e0, n, self.E_chunk(e0, n), self.SK, self.info,
                                  self.cond_work, stream)

    def assemble(self, stream=None):
        self.ctx.hdg_assemble_trace(self.SK, self.S, self.g, stream)

    def asm_setup(self, stream=None):
        self.ctx.hdg_asm_setup(self.asm_prec, self.S, self.Sinv, self.asm_info, self.asm_work, stream)

    def gmres(self, stream=None):
        self.ctx.hdg_gmres(self.asm_prec, self.S, self.Sinv, self.g, self.m, self.dUhat, self.hist,
                           self.gm_work, stream)

    def recover(self, stream=None):
        for e0, n in self.chunks:
            self.ctx.hdg_recover_interior(self.prec, e0, n, self.E_chunk(e0, n), self.dUhat, self.dQU, stream)

    def run(self, stream=None):
        """The whole hot path for one Newton step."""
        self.residual_jacobian(stream)
        self.condense(stream)
        self.assemble(stream)
        self.asm_setup(stream)
        self.gmres(stream)
        self.recover(stream)
