"""Benchmark of the HDG hot path on one MI355X.

Default workload: the 12^3 periodic supersonic Taylor-Green vortex at p = 4
(1728 hexahedra, n = 2500 interior and f = 750 trace unknowns per element),
the largest configuration that fits one GPU, processed in chunks of 256
elements.  One step = one Newton step of the whole hot path, all inputs
resident in HBM: element residuals and Jacobians, condensation, trace
assembly, additive-Schwarz set-up (FP32 inverses), 50 GMRES iterations and
interior recovery.  The headline `value` is the condensation rate
N_e / (T(hdg_condense over all chunks) + T(hdg_assemble_trace)) of the FP64
path, from HIP events on the stream the kernels run on (median over the timed
steps); the whole-step rate, the step replayed from the library's HIP graph,
the mixed-precision path (FP32 factorisation, one FP64-residual refinement,
FP64 Schur product) with its differences from the FP64 path, the face matvec
(HBM) and the CPU oracle on a bounded sample are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
PEAK_HBM_GBPS = 8000.0    # MI355X HBM3E


def condense_flops_per_element(n, f):
    """Dense condensation as specified: LU of A (2n^3/3), solve with n x (f+1)
    right-hand sides (2n^2(f+1)), Schur product C X (2fn(f+1))."""
    return 2.0 * n ** 3 / 3.0 + 2.0 * n * n * (f + 1) + 2.0 * f * n * (f + 1)


# Column fields of A that can be nonzero in each row field (fields q_(c,j) = 3c+j,
# u_c = 15+c): R_q couples q_(c,j) to itself and to u_c; R_u couples u_c to all
# of u and to the gradients its fluxes read (q_0 through the artificial
# viscosity for the mass row, the velocity gradients for the momentum rows, all
# of q for the energy row).  109 of the 400 N_p x N_p blocks.
A_NONZERO_BLOCKS = 15 * 2 + (5 + 3) + 3 * (5 + 12) + (5 + 15)


def mixed_flops_per_element(n, f, refine=1):
    """Mixed condensation, (FP32 flops, FP64 flops): FP32 LU (2n^3/3), FP32
    forward and back substitution of n x (f+1) right-hand sides (2n^2(f+1)),
    per refinement step an FP64 residual [B|R_qu] - A X over A's structurally
    nonzero blocks (2 * 109 N_p^2 (f+1)) and an FP32 solve (2n^2(f+1)); the
    FP64 Schur product (2fn(f+1))."""
    Np = n // 20
    f32 = 2.0 * n ** 3 / 3.0 + 2.0 * n * n * (f + 1) * (1 + refine)
    f64 = 2.0 * A_NONZERO_BLOCKS * Np * Np * (f + 1) * refine + 2.0 * f * n * (f + 1)
    return f32, f64


def measured_traffic(name):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (profiles/<name>.json), or None when the kernel sources it was taken on
    have changed since (their SHA-256 no longer matches)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for src, digest in rec["sources_sha256"].items():
        with open(os.path.join(ROOT, src), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != digest:
                return None
    return rec["bytes_per_launch"]


def calibration_copy(torch):
    """A plain 1 GiB device-to-device copy: the known-size reference that scales
    the FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    src = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def measure_peaks(torch, hdg):
    """Attainable peaks measured with the library's probes (hdg_peak_mfma,
    hdg_peak_copy): back-to-back FP64 and FP32 16x16x4 matrix-core products
    from registers on every SIMD, and a 1 GiB streaming copy (read + write).
    Best of five timed calls each; the probe results are checked exactly."""
    stream = torch.cuda.current_stream()

    def best_ms(fn, reps=5):
        fn()
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        return min(times)

    out = {}
    n_wg = 256 * 8  # eight workgroups of four waves per CU
    for bits, iters in ((64, 4000), (32, 8000)):
        sink = torch.empty(n_wg * 256, dtype=torch.float64 if bits == 64 else torch.float32, device="cuda")
        ms = best_ms(lambda: hdg.hdg_peak_mfma(bits, n_wg, iters, 1.0, sink))
        if not bool((sink == 128.0 * iters).all().item()):
            raise RuntimeError(f"hdg_peak_mfma FP{bits} returned a wrong sum")
        out[f"fp{bits}_mfma_tflops"] = n_wg * 4 * iters * 8 * 2048 / (ms * 1e-3) / 1e12
        del sink
    nbytes = 1 << 32  # 4 GiB, far beyond the 256 MB last-level cache
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    ms = best_ms(lambda: hdg.hdg_peak_read(src, sink))
    out["read_gbps"] = nbytes / (ms * 1e-3) / 1e9
    dst = torch.empty_like(src)
    ms = best_ms(lambda: hdg.hdg_peak_copy(src, dst))
    if not torch.equal(src, dst):
        raise RuntimeError("hdg_peak_copy did not copy")
    out["copy_gbps"] = 2.0 * nbytes / (ms * 1e-3) / 1e9
    del src, dst, sink
    out["what"] = ("hdg_peak_mfma: 2048 workgroups x 4 waves x 8 independent 16x16x4 products per iteration, "
                   "operands and accumulators in VGPRs; hdg_peak_read: 4 GiB in 64 KB chunks per workgroup, four "
                   "16-byte nontemporal loads in flight per lane; hdg_peak_copy: the same walk over 4 GiB, GB/s "
                   "counts read + write; best of 5")
    return out


def matvec_bytes(ctx):
    """Algorithmic bytes of y = S x: S's blocks read once (not the padding that
    starts each block on a 128-byte line), block-sparse indices, x read once, y
    written once."""
    import numpy as np
    rp, col, fo = (ctx.layout[k] for k in ("bsr_row_ptr", "bsr_col", "face_off"))
    b = np.diff(fo).astype(np.float64)
    rows = np.repeat(np.arange(ctx.n_face), np.diff(rp))
    s_entries = float(np.sum(b[rows] * b[col]))
    return 8.0 * s_entries + 4.0 * len(col) + 4.0 * (ctx.n_face + 1) + 2.0 * 8.0 * ctx.N_uh


def host_cpu():
    """(logical CPUs seen by the process, CPU model) of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(wl, seconds=15.0):
    """The oracle (plain C element systems + textbook LU condensation) on the
    host cores, timed on a sample of the benchmark's elements: the element
    systems are built first, then only their condensation is timed (the
    quantity of the headline rate), on all allowed cores and on one core."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    O.build()
    sz = O.Sizes(wl.mesh)
    nproc, model = host_cpu()
    cores = max(1, min(16, nproc))  # a one-GPU share of the host

    def build(e):
        return O.element_system(wl, e, sz)

    t0 = time.perf_counter()
    E0 = build(0)
    t_sys = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.condense(E0, sz.n(0))
    t_one = max(time.perf_counter() - t0, 1e-3)
    # one core: as many whole elements as fit in about a third of the budget
    k1 = max(1, min(wl.mesh.n_elem, int((seconds / 3.0) / t_one)))
    systems = [E0] + [build(e) for e in range(1, k1)]
    t0 = time.perf_counter()
    for e in range(k1):
        O.condense(systems[e], sz.n(e))
    t1 = time.perf_counter() - t0
    # all cores: whole waves of `cores` elements in the remaining budget
    waves = max(1, int((2.0 * seconds / 3.0) / t_one))
    count = min(wl.mesh.n_elem, cores * waves)
    with ThreadPoolExecutor(max_workers=cores) as ex:
        systems = list(ex.map(build, range(count)))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(lambda e: O.condense(systems[e], sz.n(e)), range(count)))
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "elements/s", "cores": cores, "kind": "oracle",
            "sample": f"condensation (LU of A, solve for [B | R_qu], Schur product) of elements 0..{count - 1} "
                      f"({count} of {wl.mesh.n_elem}) of the same workload on {cores} threads, {dt:.1f} s wall; "
                      f"element systems built beforehand ({t_sys:.1f} s each on one core), not timed",
            "one_core": {"value": k1 / t1, "unit": "elements/s", "elements": k1, "seconds": t1},
            "host": {"nproc": nproc, "model": model}}


def measured_record(name):
    """A committed counter summary (profiles/<name>.json) while the kernel
    sources it was taken on are unchanged (their SHA-256 still matches)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for src, digest in rec["sources_sha256"].items():
        with open(os.path.join(ROOT, src), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != digest:
                return None
    return rec


WORKLOAD_TAG = {1: "tgv8_p3", 3: "bl2000_p234", 4: "tgv12_p4"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed Newton steps (each path)")
    ap.add_argument("--warmup", type=int, default=3, help="untimed Newton steps before timing (each path)")
    ap.add_argument("--config", type=int, default=4, choices=(1, 3, 4),
                    help="4 (default): 12^3 p=4 supersonic TGV, chunks of 256, GMRES(50) with FP32 Schwarz; "
                         "1: 8^3 p=3 supersonic TGV with AV, GMRES(30) with FP64 Schwarz; "
                         "3: 2000 wall-stretched hexahedra with p in {2,3,4}")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay timing")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--matvec-reps", type=int, default=100)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default 128-row update tiles")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU's partition only (--gpus {args.gpus} requested); "
              "element-partition sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("bench.py: --steps must be at least 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth

    peaks = measure_peaks(torch, hdg)
    print(f"[bench] measured peaks: FP64 matrix {peaks['fp64_mfma_tflops']:.1f} TFLOP/s, FP32 matrix "
          f"{peaks['fp32_mfma_tflops']:.1f} TFLOP/s, read {peaks['read_gbps']:.0f} GB/s, copy "
          f"{peaks['copy_gbps']:.0f} GB/s", file=sys.stderr, flush=True)
    big = args.config == 4
    wl = synth.config(args.config)
    chunk = 256 if big else None
    asm_fp64 = hdg.HDG_MIXED if big else hdg.HDG_FP64  # the p=4 workload uses FP32 Schwarz blocks throughout
    print(f"[bench] workload {wl.name}: building context", file=sys.stderr, flush=True)
    st = pipeline.NewtonStep(wl, prec=hdg.HDG_FP64, asm_prec=asm_fp64, chunk=chunk)
    ctx = st.ctx
    ne = ctx.n_elem
    ns = [int(v) for v in ctx.layout["elem_n"]]
    fs = [int(v) for v in ctx.layout["elem_f"]]
    n, f = ns[0], fs[0]
    degrees = sorted(set(int(v) for v in wl.mesh.elem_p))
    p = degrees[0] if len(degrees) == 1 else "-".join(str(d) for d in degrees)
    stream = torch.cuda.current_stream()
    phases = ["residual_jacobian", "condense", "assemble", "asm_setup", "gmres", "recover"]

    def stepper(obj):
        def step(events=None):
            for i, ph in enumerate(phases):
                if events is not None:
                    events[i].record(stream)
                getattr(obj, ph)()
            if events is not None:
                events[-1].record(stream)
        return step

    def timed(run_step, label):
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            run_step(evs[k])
            if (k + 1) % 5 == 0 or k + 1 == args.steps:
                torch.cuda.synchronize()
                print(f"[bench] {label}: {k + 1}/{args.steps} timed steps", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = np.array([[evs[k][i].elapsed_time(evs[k][i + 1]) for i in range(len(phases))]
                        for k in range(args.steps)])
        med = {ph: float(np.median(per[:, i])) for i, ph in enumerate(phases)}
        mins = {ph: float(per[:, i].min()) for i, ph in enumerate(phases)}
        ic, ia = phases.index("condense"), phases.index("assemble")
        cond_asm = per[:, ic] + per[:, ia]
        return dict(ms_step=1e3 * wall / args.steps, phase_ms=med, phase_ms_min=mins,
                    condense_ms=float(np.median(per[:, ic])), condense_ms_min=float(per[:, ic].min()),
                    cond_asm_ms=float(np.median(cond_asm)), cond_asm_ms_min=float(cond_asm.min()))

    def timed_graph(obj, label):
        reps = max(3, args.steps // 4)
        graph = obj.capture()
        graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            graph.replay()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        graph.close()
        print(f"[bench] {label} graph replay: {ms:.2f} ms/step ({reps} replays)", file=sys.stderr, flush=True)
        return {"ms_per_step": ms, "replays": reps}

    def check(obj, what):
        if not np.all(obj.info.cpu().numpy() == 0) or not np.all(obj.asm_info.cpu().numpy() == 0):
            raise RuntimeError(f"zero pivot reported in the {what} warm-up")

    def warm(step, label):
        for w in range(args.warmup):
            step()
            torch.cuda.synchronize()
            print(f"[bench] {label}: warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    # tile shape of the LU's trailing update, per size of system, chosen by measurement
    tiles = None
    if not args.no_autotune:
        table = pipeline.autotune_update_tiles(st, log=lambda m: print(m, file=sys.stderr, flush=True))
        tiles = {str(k): {"rows": v[0], "ms": {str(r): t for r, t in v[1].items()}} for k, v in table.items()}

    # ---------------------------------------------------------------- FP64 path
    step = stepper(st)
    warm(step, "FP64")
    check(st, "FP64")
    r64 = timed(step, "FP64")
    print(f"[bench] FP64: {r64['ms_step']:.2f} ms/step, condensation + assembly {r64['cond_asm_ms']:.2f} ms",
          file=sys.stderr, flush=True)
    graph64 = None if args.no_graph else timed_graph(st, "FP64")
    S64, g64, d64 = (st.S.clone(), st.g.clone(), st.dUhat.clone()) if not args.no_mixed else (None, None, None)

    # face matvec roofline (HBM): algorithmic bytes / kernel time, alternating buffers
    x0 = torch.as_tensor(wl.x, dtype=torch.float64, device="cuda")
    xs = [x0, x0.clone()]
    ys = [torch.empty_like(x0) for _ in range(2)]
    for _ in range(3):
        ctx.hdg_face_matvec(st.S, xs[0], ys[0])
    reps = max(10, args.matvec_reps)
    mv_ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    mv_ev[0].record(stream)
    for r in range(reps):
        ctx.hdg_face_matvec(st.S, xs[r % 2], ys[r % 2])
        mv_ev[r + 1].record(stream)
    torch.cuda.synchronize()
    mv_all = np.array([mv_ev[r].elapsed_time(mv_ev[r + 1]) for r in range(reps)])
    mv_ms = float(np.median(mv_all))
    mv_bytes = matvec_bytes(ctx)
    mv_gbps = mv_bytes / (mv_ms * 1e-3) / 1e9

    # -------------------------------------------------------------- mixed path
    mixed = None
    if not args.no_mixed:
        stm = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, refine_steps=1, ctx=ctx, chunk=chunk,
                                  share=st if big else None)
        step_mixed = stepper(stm)
        warm(step_mixed, "mixed")
        check(stm, "mixed")
        rm = timed(step_mixed, "mixed")
        print(f"[bench] mixed: {rm['ms_step']:.2f} ms/step, condensation + assembly {rm['cond_asm_ms']:.2f} ms",
              file=sys.stderr, flush=True)
        graphm = None if args.no_graph else timed_graph(stm, "mixed")
        relnorm = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        mfl = [mixed_flops_per_element(a, b, 1) for a, b in zip(ns, fs)]
        f32tot, f64tot = sum(x[0] for x in mfl), sum(x[1] for x in mfl)
        t_cm = rm["condense_ms"] * 1e-3
        t_peak = f32tot / (PEAK_FP32_TFLOPS * 1e12) + f64tot / (PEAK_FP64_TFLOPS * 1e12)
        t_peak_m = f32tot / (peaks["fp32_mfma_tflops"] * 1e12) + f64tot / (peaks["fp64_mfma_tflops"] * 1e12)
        mixed = {
            "value": ne / (rm["cond_asm_ms"] * 1e-3), "unit": "elements/s",
            "ms_per_step": rm["ms_step"], "step_elements_per_s": ne / (rm["ms_step"] * 1e-3),
            "graph": graphm, "phase_ms": rm["phase_ms"], "phase_ms_min": rm["phase_ms_min"],
            "condense_ms": rm["condense_ms"], "refine_steps": 1,
            "schwarz": "element-block, FP32 inverses",
            "rel_diff_vs_fp64_path": {"S": relnorm(stm.S, S64), "g": relnorm(stm.g, g64),
                                      "dUhat_fixed_m": relnorm(stm.dUhat, d64)},
            "roofline": {"bound": "mfma", "time_at_peak_ms": 1e3 * t_peak, "frac": t_peak / t_cm,
                         "time_at_measured_peak_ms": 1e3 * t_peak_m, "frac_of_measured_peak": t_peak_m / t_cm,
                         "algorithmic": f"{f32tot:.4e} FP32 + {f64tot:.4e} FP64 flop over {ne} elements "
                                        f"(peaks {PEAK_FP32_TFLOPS} / {PEAK_FP64_TFLOPS} TFLOP/s; the FP64 "
                                        f"refinement residual counts A's {A_NONZERO_BLOCKS} of 400 nonzero blocks)"},
        }

    # the mixed step with streamed element systems: one chunk of E at a time, X retained
    streamed = None
    if not args.no_mixed and chunk is not None:
        ref_dU, ref_dQU = stm.dUhat.clone(), stm.dQU.clone()
        sts = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, refine_steps=1, ctx=ctx, chunk=chunk, share=stm,
                                  stream_E=True)
        step_s = stepper(sts)
        step_s()
        torch.cuda.synchronize()
        same = bool(torch.equal(sts.dUhat, ref_dU) and torch.equal(sts.dQU, ref_dQU))
        reps_s = max(2, args.steps // 4)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps_s)]
        for a, b in evs:
            a.record(stream)
            step_s()
            b.record(stream)
        torch.cuda.synchronize()
        ms_s = float(np.median([a.elapsed_time(b) for a, b in evs]))
        eo = ctx.layout["E_off"]
        streamed = {"ms_per_step": ms_s, "reps": reps_s, "identical_to_resident_mixed_step": same,
                    "E_bytes_streamed": 8 * max(int(eo[e0 + n] - eo[e0]) for e0, n in sts.chunks),
                    "X_bytes": 8 * int(ctx.layout["x_off"][-1]), "E_bytes_resident": 8 * int(eo[-1]),
                    "what": "each chunk's systems formed, condensed and X = A^-1[B | R_qu] kept (hdg_store_x); "
                            "recovery from X (hdg_recover_interior_x)"}
        print(f"[bench] mixed, streamed systems: {ms_s:.2f} ms/step, identical {same}", file=sys.stderr, flush=True)
        del sts

    # all-FP32 condensation (no refinement): its time and its error, reported beside the mixed path
    fast = None
    if not args.no_mixed:
        stf = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED_FAST, ctx=ctx, chunk=chunk, share=st if big else stm)
        reps_f = max(2, min(3, args.steps))
        times = []
        for rep in range(reps_f + 1):
            stf.residual_jacobian()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            stf.condense()
            stf.assemble()
            b.record(stream)
            torch.cuda.synchronize()
            if rep:
                times.append(a.elapsed_time(b))
        if stf.info.any().item():
            raise RuntimeError("zero pivot reported by the all-FP32 condensation")
        relnorm = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        t_f = float(np.median(times))
        fast = {"value": ne / (t_f * 1e-3), "unit": "elements/s", "condense_assemble_ms": t_f, "reps": reps_f,
                "rel_diff_vs_fp64_path": {"S": relnorm(stf.S, S64), "g": relnorm(stf.g, g64)},
                "what": "whole bordered system factored in FP32, Schur complement from FP32 trailing updates with "
                        "FP32 accumulation, no refinement (HDG_MIXED_FAST); not accurate to 1e-10"}
        print(f"[bench] all-FP32 condensation + assembly: {t_f:.2f} ms, S rel diff {fast['rel_diff_vs_fp64_path']['S']:.2e}",
              file=sys.stderr, flush=True)
        del stf

    # condensation roofline (FP64 matrix cores): dense algorithmic flops / hdg_condense time
    fl = sum(condense_flops_per_element(a, b) for a, b in zip(ns, fs))
    t_cond = r64["condense_ms"] * 1e-3
    achieved = fl / t_cond / 1e12
    tag = WORKLOAD_TAG[args.config]
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "peak_measured": peaks["fp64_mfma_tflops"], "frac_of_measured_peak": achieved / peaks["fp64_mfma_tflops"],
            "traffic": measured_traffic(f"condense_fp64_{tag}_hbm"),
            "kernel": "hdg_condense (all chunks; per pair of 128-column blocks k_panel, k_half, k_crows, k_rowperm, "
                      "k_inv128, k_blocku, k_update; then k_extract)",
            "algorithmic": f"{fl:.4e} flop over {ne} elements (LU 2n^3/3 + solve 2n^2(f+1) + Schur 2fn(f+1) per "
                           f"element), median hdg_condense time {r64['condense_ms']:.2f} ms"}
    mf = measured_record(f"condense_fp64_{tag}_mfma")
    if mf is not None:
        roof["mfma_counters"] = {k: mf[k] for k in ("mfma_flops_per_launch", "mfma_busy_frac") if k in mf}
    out = {
        "metric": "HDG condensed elements/s, FP64 vs mixed @1e-10 rel; face-matvec GB/s",
        "value": ne / (r64["cond_asm_ms"] * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "elements": ne, "p": p,
                   "n_interior": n if len(degrees) == 1 else f"{min(ns)}-{max(ns)}",
                   "f_trace": f if len(degrees) == 1 else f"{min(fs)}-{max(fs)}",
                   "chunk": chunk or ne, "batches": [c for _, c in st.chunks], "gmres_iterations": st.m,
                   "schwarz": "element-block, " + ("FP32 inverses" if big else "FP64"), "precision": "FP64",
                   "step": f"residual+Jacobian, condensation, assembly, Schwarz set-up, GMRES({st.m}), recovery",
                   "value_is": "N_e / median(T(hdg_condense, all chunks) + T(hdg_assemble_trace))",
                   "update_tiles": tiles},
        "step_elements_per_s": ne / (r64["ms_step"] * 1e-3),
        "condense_ms": r64["condense_ms"],
        "condense_assemble_ms": r64["cond_asm_ms"],
        "condense_assemble_ms_min": r64["cond_asm_ms_min"],
        "graph": graph64,
        "phase_ms": r64["phase_ms"],
        "phase_ms_min": r64["phase_ms_min"],
        "roofline": roof,
        "roofline_matvec": {"bound": "hbm", "achieved": mv_gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                            "frac": mv_gbps / PEAK_HBM_GBPS, "peak_measured": peaks["read_gbps"],
                            "frac_of_measured_peak": mv_gbps / peaks["read_gbps"],
                            "traffic": measured_traffic(f"matvec_{tag}_hbm"),
                            "kernel": "k_matvec", "ms_median": mv_ms, "ms_min": float(mv_all.min()),
                            "reps": reps, "algorithmic_bytes": mv_bytes},
        "mixed": mixed,
        "mixed_fast": fast,
        "mixed_streamed": streamed,
        "measured_peaks": peaks,
    }
    calibration_copy(torch)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
