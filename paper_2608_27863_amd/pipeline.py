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

from .hdg import HDG_FP64, HDG_MIXED, Context, HDGError


class NewtonStep:
    def __init__(self, wl, prec=HDG_FP64, refine_steps=1, asm_prec=None, chunk=None, m=None,
                 ctx=None, device="cuda", share=None, stream_E=False):
        """share: another NewtonStep on the same context whose device buffers are
        reused where shape and type agree (the two steps then overwrite each
        other's results; useful when the element systems are large).
        stream_E (HDG_MIXED only): one chunk's element systems at a time.  E
        holds the largest chunk; each chunk is assembled, condensed and its
        X = A^{-1}[B | R_qu] copied to a resident store (hdg_store_x) before the
        next chunk reuses E; the recovery reads that store
        (hdg_recover_interior_x).  At p = 4 that is 15 MB per element instead
        of the system's 84.5 MB."""
        import torch
        if stream_E and prec != HDG_MIXED:
            raise ValueError("stream_E needs HDG_MIXED (the recovery then reads only X)")
        self.wl = wl
        self.prec = prec
        self.refine = refine_steps
        # Schwarz inverses: FP64 with the FP64 path, FP32 otherwise
        self.asm_prec = (HDG_FP64 if prec == HDG_FP64 else HDG_MIXED) if asm_prec is None else asm_prec
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
        self.stream_E = bool(stream_E)
        if self.stream_E:
            eo = c.layout["E_off"]
            self.E = buf("E", max(int(eo[e0 + n] - eo[e0]) for e0, n in self.chunks))
            self.X = buf("X", int(c.layout["x_off"][-1]))
        else:
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
        if self.stream_E:
            return self.E[:int(o[e0 + n] - o[e0])]
        return self.E[int(o[e0]):int(o[e0 + n])]

    def _rj(self, e0, n, stream=None):
        self.ctx.hdg_local_residual_jacobian(e0, n, self.Q, self.U, self.Un, self.Uhat, self.nu,
                                             self.Ub if self.wl.mesh.face_bc.any() else None,
                                             self.E_chunk(e0, n), self.qp_work, stream)

    # the steps of the hot path
    def residual_jacobian(self, stream=None):
        """Element systems of every chunk (resident E).  With stream_E the
        systems are formed chunk by chunk inside condense()."""
        if self.stream_E:
            return
        for e0, n in self.chunks:
            self._rj(e0, n, stream)

    def condense(self, stream=None):
        for e0, n in self.chunks:
            if self.stream_E:
                self._rj(e0, n, stream)
            self.ctx.hdg_condense(self.prec, self.refine, e0, n, self.E_chunk(e0, n), self.SK, self.info,
                                  self.cond_work, stream)
            if self.stream_E:
                self.ctx.hdg_store_x(e0, n, self.E_chunk(e0, n), self.X, stream)

    def assemble(self, stream=None):
        self.ctx.hdg_assemble_trace(self.SK, self.S, self.g, stream)

    def asm_setup(self, stream=None):
        self.ctx.hdg_asm_setup(self.asm_prec, self.S, self.Sinv, self.asm_info, self.asm_work, stream)

    def gmres(self, stream=None):
        self.ctx.hdg_gmres(self.asm_prec, self.S, self.Sinv, self.g, self.m, self.dUhat, self.hist,
                           self.gm_work, stream)

    def recover(self, stream=None):
        if self.stream_E:
            self.ctx.hdg_recover_interior_x(0, self.ctx.n_elem, self.X, self.dUhat, self.dQU, stream)
            return
        # every system is resident: one launch over all elements (each element's
        # recovery is independent, so this equals the per-chunk calls bit for bit)
        self.ctx.hdg_recover_interior(self.prec, 0, self.ctx.n_elem, self.E, self.dUhat, self.dQU, stream)

    def run(self, stream=None):
        """The whole hot path for one Newton step, as one call (hdg_newton_step)."""
        if self.stream_E:
            raise ValueError("the one-call step keeps every element system resident; use run_calls")
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
        if self.stream_E:
            raise ValueError("the captured step keeps every element system resident")
        if getattr(self, "_args", None) is None:
            self._args = self.ctx.newton_args(self)
        s = stream if stream is not None else torch.cuda.Stream()
        torch.cuda.synchronize()
        graph = self.ctx.hdg_graph_capture_newton(self._args, s)
        torch.cuda.synchronize()
        return graph


class NewtonSolver:
    """Newton's method for one DIRK stage (sections 2.4-3.4) on the buffers of a
    NewtonStep: the state (Q, U, Uhat) is updated in place, the lagged state
    of the mass term is the step's Un.  Each iteration evaluates the element
    residuals and Jacobians, gathers the residual norm (eq. nonlinear-residual),
    stops once it is at most max(atol, tol * the first one), else condenses,
    assembles, sets up the Schwarz blocks, takes the reduced-basis guess
    (eq. rb-min; window of rb_max accepted corrections, 0 = no guess), runs
    GMRES from it, inserts the accepted correction into the window, recovers
    the interior correction and updates the state with the largest
    alpha in {1, 1/2, ..., 2^-10} that keeps density and pressure positive
    (eq. newton-update).  The host reads three norms and a flag per iteration;
    all arithmetic runs in libhdg's kernels."""

    def __init__(self, step, rb_max=0, tol=1e-10, atol=1e-11, maxit=8):
        import torch
        self.st = step
        ctx = step.ctx
        self.tol, self.atol, self.maxit = tol, atol, maxit
        dev = step.E.device
        self.rwork = torch.empty(ctx.workspace_size(6), dtype=torch.uint8, device=dev)
        self.norms = torch.zeros(3, dtype=torch.float64, device=dev)
        self.flag = torch.zeros(1, dtype=torch.int32, device=dev)
        self.rb_max = int(rb_max)
        self.count = self.head = 0
        if self.rb_max:
            if not 1 <= self.rb_max <= 32:
                raise ValueError("rb_max must be in 0..32")
            self.W = torch.zeros(self.rb_max * ctx.N_uh, dtype=torch.float64, device=dev)
            self.Z = torch.zeros_like(self.W)
            self.x0 = torch.zeros(ctx.N_uh, dtype=torch.float64, device=dev)
            self.rb_work = torch.empty(ctx.workspace_size(5, 0, 0, self.rb_max), dtype=torch.uint8, device=dev)

    def residual(self, stream=None):
        """Element systems at the current state and (||R_q||, ||R_u||, ||R_uh||)."""
        st, ctx = self.st, self.st.ctx
        for e0, n in st.chunks:
            ctx.hdg_local_residual_jacobian(e0, n, st.Q, st.U, st.Un, st.Uhat, st.nu,
                                            st.Ub if st.wl.mesh.face_bc.any() else None, st.E_chunk(e0, n),
                                            st.qp_work, stream)
            ctx.hdg_residual_gather(e0, n, st.E_chunk(e0, n), self.rwork, stream)
        ctx.hdg_residual_norm(self.rwork, self.norms, stream)
        return tuple(float(v) for v in self.norms.cpu())

    def pivot_failure(self):
        """None, or which factorisation met a zero or non-finite pivot (the
        device info arrays: k+1 for the k-th pivot) and in which element."""
        import torch
        st = self.st
        for what, info in (("condensation", st.info), ("Schwarz set-up", st.asm_info)):
            bad = torch.nonzero(info).flatten().cpu()
            if bad.numel():
                e = int(bad[0])
                return (f"{what}: pivot {int(info[e])} of element {e} is zero or not finite"
                        f" ({bad.numel()} element(s) affected)")
        return None

    def solve(self, stream=None):
        """Returns the history [(||R_q||, ||R_u||, ||R_uh||, alpha, GMRES history), ...]."""
        import math
        st, ctx = self.st, self.st.ctx
        hist, f0 = [], None
        for it in range(self.maxit + 1):
            nr = self.residual(stream)
            fn = math.sqrt(sum(v * v for v in nr))
            f0 = fn if f0 is None else f0
            if fn <= max(self.atol, self.tol * f0) or it == self.maxit:
                hist.append((*nr, None, None))
                break
            st.condense(stream)
            st.assemble(stream)
            st.asm_setup(stream)
            failed = self.pivot_failure()
            if failed:
                raise HDGError(f"Newton iteration {it}: {failed}")
            if self.rb_max and self.count:
                ctx.hdg_rb_guess(self.count, self.W, self.Z, st.g, self.x0, self.rb_work, stream)
                ctx.hdg_gmres_x0(st.asm_prec, st.S, st.Sinv, st.g, self.x0, st.m, st.dUhat, st.hist, st.gm_work,
                                 stream)
            else:
                st.gmres(stream)
            if self.rb_max:
                self.count, self.head = ctx.hdg_rb_insert(st.S, st.dUhat, self.rb_max, self.count, self.head,
                                                          self.W, self.Z, stream)
            st.recover(stream)
            alpha = 1.0
            while True:
                ctx.hdg_state_admissible(alpha, st.U, st.dQU, self.flag, stream)
                if int(self.flag.cpu()[0]) == 0 or alpha <= 2.0 ** -10:
                    break
                alpha *= 0.5
            ctx.hdg_state_update(alpha, st.dQU, st.dUhat, st.Q, st.U, st.Uhat, stream)
            hist.append((*nr, alpha, st.hist.cpu().numpy().copy()))
        return hist


def alexander_dirk():
    """Alexander's three-stage, third-order, L-stable DIRK: (A, b) with
    a_ii = gamma, the root near 0.4359 of gamma^3 - 3 gamma^2 + 3 gamma / 2 - 1/6,
    a_21 = (1 - gamma)/2, last row b = (-(6g^2 - 16g + 1)/4, (6g^2 - 20g + 5)/4, g);
    and the coefficients d = A^{-1}, e = b^T d of eqs. dirk-stage, dirk-update."""
    g = 0.4358
    for _ in range(50):  # Newton on the cubic
        g -= (g ** 3 - 3 * g ** 2 + 1.5 * g - 1.0 / 6.0) / (3 * g ** 2 - 6 * g + 1.5)
    b = [-(6 * g * g - 16 * g + 1) / 4, (6 * g * g - 20 * g + 5) / 4, g]
    A = [[g, 0.0, 0.0], [(1 - g) / 2, g, 0.0], list(b)]
    # inverse of the lower-triangular A by forward substitution, column by column
    d = [[0.0] * 3 for _ in range(3)]
    for col in range(3):
        for r in range(3):
            s = (1.0 if r == col else 0.0) - sum(A[r][k] * d[k][col] for k in range(r))
            d[r][col] = s / A[r][r]
    e = [sum(b[i] * d[i][j] for i in range(3)) for j in range(3)]
    return A, b, d, e


class DirkStepper:
    """One time step of the three-stage DIRK (eqs. dirk-stage, dirk-update) on a
    NewtonSolver's buffers: stage i sets the lagged state
    Un <- U^n - sum_{j<i} (d_ij / d_ii)(U^{n,j} - U^n) (so that the residual's
    d_ii M (U - Un) is the stage's mass term) and solves from the previous
    stage's state; then U <- (1 - sum_j e_j) U^n + sum_j e_j U^{n,j}, keeping Q
    and Uhat of the last stage (the tableau is stiffly accurate: e = (0, 0, 1)).
    The context's alpha must be d_ii.  With `av` (hdg_av_field parameters:
    c_av, h_m, eps, s_max, rho_min, p_min, smooth_iters) the artificial
    viscosity is recomputed from the state at the start of each step and held
    fixed during it (lagged)."""

    def __init__(self, solver, av=None):
        import torch
        self.solver = solver
        st = solver.st
        self.av = av
        if av is not None:
            self.av_work = torch.empty(st.ctx.workspace_size(7), dtype=torch.uint8, device=st.E.device)
        self.A, self.b, self.d, self.e = alexander_dirk()
        if abs(st.wl.alpha - self.d[0][0]) > 1e-12 * self.d[0][0]:
            raise ValueError("the context's alpha must equal d_ii = 1 / gamma of the tableau")
        self.Un = torch.empty_like(st.U)
        self.stages = [torch.empty_like(st.U) for _ in range(3)]

    def step(self, stream=None):
        st, ctx, d, e = self.solver.st, self.solver.st.ctx, self.d, self.e
        if self.av is not None:
            ctx.hdg_av_field(self.av, st.U, st.Q, st.nu, self.av_work, stream=stream)
        ctx.hdg_lincomb([st.U], [1.0], self.Un, stream)
        hists = []
        for i in range(3):
            coefs = [1.0 + sum(d[i][j] / d[i][i] for j in range(i))] + [-d[i][j] / d[i][i] for j in range(i)]
            ctx.hdg_lincomb([self.Un] + self.stages[:i], coefs, st.Un, stream)
            hists.append(self.solver.solve(stream))
            ctx.hdg_lincomb([st.U], [1.0], self.stages[i], stream)
        ctx.hdg_lincomb([self.Un] + self.stages, [1.0 - sum(e)] + list(e), st.U, stream)
        return hists


def autotune_update_tiles(step, candidates=(128, 256), reps=2, schwarz=True, log=None):
    """Choose the trailing-update tile of the blocked LU by measurement on the
    device: for each size of element system in the step (n = 20 N_p), time
    hdg_condense of that size's chunks with each candidate tile height (the
    element systems are rebuilt by hdg_local_residual_jacobian before every
    timed run, since condensation overwrites them), keep the fastest in the
    context (hdg_set_update_tile) and return the table {n: (rows, {rows: ms})}.
    With `schwarz`, the Schwarz inversion systems (size f rounded up to a
    multiple of 4) are tuned on hdg_asm_setup after one whole step."""
    import torch
    ctx = step.ctx
    s = torch.cuda.current_stream()
    sizes = {}
    for e0, n in step.chunks:
        sizes.setdefault(int(ctx.layout["elem_n"][e0]), []).append((e0, n))
    table = {}

    def timed(fn):
        best = None
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            fn()
            b.record(s)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        return best

    for nsz, chunks in sorted(sizes.items()):
        times = {}
        for rows in candidates:
            ctx.hdg_set_update_tile(nsz, rows)

            def run():
                for e0, n in chunks:
                    ctx.hdg_condense(step.prec, step.refine, e0, n, step.E_chunk(e0, n), step.SK, step.info,
                                     step.cond_work)
            ms = None
            for _ in range(reps):
                for e0, n in chunks:
                    ctx.hdg_local_residual_jacobian(e0, n, step.Q, step.U, step.Un, step.Uhat, step.nu,
                                                    step.Ub if step.wl.mesh.face_bc.any() else None,
                                                    step.E_chunk(e0, n), step.qp_work)
                t = timed(run)
                ms = t if ms is None else min(ms, t)
            times[rows] = ms
        best = min(times, key=times.get)
        ctx.hdg_set_update_tile(nsz, best)
        table[nsz] = (best, times)
        if log:
            log(f"[autotune] element systems n={nsz}: " + ", ".join(f"{r} rows {t:.2f} ms" for r, t in times.items())
                + f" -> {best}")
    if schwarz:
        step.run_calls()
        torch.cuda.synchronize()
        maxf = int(max(ctx.layout["elem_f"]))
        m = (maxf + 3) & ~3  # size of the Schwarz inversion systems
        times = {}
        for rows in candidates:
            ctx.hdg_set_update_tile(m, rows)
            times[rows] = timed(lambda: step.asm_setup())
        best = min(times, key=times.get)
        ctx.hdg_set_update_tile(m, best)
        table[m] = (best, times)
        if log:
            log(f"[autotune] Schwarz systems m={m}: " + ", ".join(f"{r} rows {t:.2f} ms" for r, t in times.items())
                + f" -> {best}")
    return table
