"""One Newton step of the HDG hot path on the GPU, as a sequence of libhdg calls.

Allocates the device buffers (torch) and issues, on one stream:
  hdg_local_residual_jacobian (per chunk) -> hdg_condense (per chunk)
  -> hdg_assemble_trace -> hdg_asm_setup -> hdg_gmres -> hdg_recover_interior,
either call by call or as one hdg_newton_step, or replayed from a HIP graph the
library captures (hdg_graph_capture_newton).  No arithmetic happens here;
every step runs in libhdg's kernels.
"""
from __future__ import annotations

import numpy as np

from .hdg import HDG_FP64, HDG_MIXED, Context


class NewtonStep:
    def __init__(self, wl, prec=HDG_FP64, refine_steps=1, asm_prec=None, chunk=None, m=None,
                 ctx=None, device="cuda", share=None):
        """share: another NewtonStep on the same context whose device buffers are
        reused where shape and type agree (the two steps then overwrite each
        other's results; useful when the element systems are large)."""
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
        # size buckets: a mesh whose degrees form a few contiguous runs (elements
        # numbered by degree) is split at the run boundaries, one size of
        # element system per batch of launches
        ep = np.asarray(wl.mesh.elem_p)
        cuts = [0] + [int(i) + 1 for i in np.nonzero(ep[1:] != ep[:-1])[0]] + [ne]
        if 2 < len(cuts) <= 5:
            self.chunks = []
            for lo, hi in zip(cuts[:-1], cuts[1:]):
                for a in range(lo, hi, self.chunk):
                    self.chunks.append((a, min(self.chunk, hi - a)))
        f64 = dict(dtype=torch.float64, device=device)

        def buf(name, numel, dtype=torch.float64, zero=False):
            old = getattr(share, name, None) if share is not None else None
            if old is not None and old.dtype == dtype and old.numel() >= numel:
                return old
            return (torch.zeros if zero else torch.empty)(numel, dtype=dtype, device=device)

        def inp(name, a):
            old = getattr(share, name, None) if share is not None else None
            return old if old is not None else torch.as_tensor(np.ascontiguousarray(a), **f64)

        self.Q, self.U, self.Un = inp("Q", wl.Q), inp("U", wl.U), inp("Un", wl.Un)
        self.Uhat, self.nu, self.Ub = inp("Uhat", wl.Uhat), inp("nu", wl.nu), inp("Ub", wl.Ub)
        self.E = buf("E", int(c.layout["E_off"][-1]))
        qp = max(c.workspace_size(0, HDG_FP64, e0, n) for e0, n in self.chunks)
        self.qp_work = buf("qp_work", qp, torch.uint8)
        cw = max(c.workspace_size(1, prec, e0, n) for e0, n in self.chunks)
        self.cond_work = buf("cond_work", cw, torch.uint8)
        self.SK = buf("SK", int(c.layout["SK_off"][-1]))
        self.info = buf("info", ne, torch.int32, zero=True)
        self.S = buf("S", int(c.layout["bsr_val_off"][-1]))
        self.g = buf("g", c.N_uh)
        sdt = torch.float64 if self.asm_prec == HDG_FP64 else torch.float32
        self.Sinv = buf("Sinv", int(c.layout["asm_off"][-1]), sdt)
        self.asm_info = buf("asm_info", ne, torch.int32, zero=True)
        self.asm_work = buf("asm_work", c.workspace_size(2, self.asm_prec), torch.uint8)
        self.gm_work = buf("gm_work", c.workspace_size(4, self.asm_prec, 0, self.m), torch.uint8)
        self.dUhat = buf("dUhat", c.N_uh)
        self.hist = torch.empty(self.m + 1, **f64)
        self.dQU = buf("dQU", 20 * int(c.layout["node_off"][-1]))

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
        """The whole hot path for one Newton step, as one call (hdg_newton_step)."""
        if getattr(self, "_args", None) is None:
            self._args = self.ctx.newton_args(self)
        self.ctx.hdg_newton_step(self._args, stream)

    def run_calls(self, stream=None):
        """The same step issued call by call from here."""
        self.residual_jacobian(stream)
        self.condense(stream)
        self.assemble(stream)
        self.asm_setup(stream)
        self.gmres(stream)
        self.recover(stream)

    def capture(self, stream=None):
        """The whole Newton step captured in a HIP graph by the library
        (hdg_graph_capture_newton) on `stream`, a created stream (a new one when
        None).  Blocking.  graph.replay(stream) reruns the step on the current
        contents of the input buffers; nothing is allocated or synchronised
        inside."""
        import torch
        if getattr(self, "_args", None) is None:
            self._args = self.ctx.newton_args(self)
        s = stream if stream is not None else torch.cuda.Stream()
        torch.cuda.synchronize()
        graph = self.ctx.hdg_graph_capture_newton(self._args, s)
        torch.cuda.synchronize()
        return graph
