"""Benchmark of the HDG hot path on one MI355X.

One step = one Newton step of the whole hot path on the 8^3 periodic
supersonic Taylor-Green workload at p = 3 (512 hexahedra, n = 1280 interior and
f = 480 trace unknowns per element): element residuals and Jacobians,
condensation, trace assembly, additive-Schwarz set-up, 30 GMRES iterations and
interior recovery, all inputs resident in HBM.  The FP64 step is the headline
figure; the mixed-precision step (FP32 factorisation, one FP64-residual
refinement, FP64 Schur product, FP32 Schwarz inverses) is timed on the same
workload beside it, with its differences from the FP64 step.

Prints one JSON line: whole-step throughput in elements/s, the condensation
roofline (FP64 matrix cores), the face-matvec roofline (HBM), the mixed step,
and the CPU oracle timed on a bounded sample of the same workload.
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


def mixed_flops_per_element(n, f, refine=1):
    """Mixed condensation as specified, (FP32 flops, FP64 flops): FP32 LU
    (2n^3/3), FP32 forward and back substitution of n x (f+1) right-hand sides
    (2n^2(f+1)), per refinement step a dense FP64 residual (2n^2(f+1)) and an
    FP32 solve (2n^2(f+1)); the FP64 Schur product (2fn(f+1))."""
    f32 = 2.0 * n ** 3 / 3.0 + 2.0 * n * n * (f + 1) * (1 + refine)
    f64 = 2.0 * n * n * (f + 1) * refine + 2.0 * f * n * (f + 1)
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


def matvec_bytes(ctx):
    """Algorithmic bytes of y = S x: S read once, block-sparse indices, x read
    once, y written once."""
    import numpy as np
    vo = ctx.layout["bsr_val_off"]
    nnzb = len(ctx.layout["bsr_col"])
    return 8.0 * float(vo[-1]) + 4.0 * nnzb + 4.0 * (ctx.n_face + 1) + 2.0 * 8.0 * ctx.N_uh


def cpu_baseline(wl, seconds=15.0):
    """The oracle (plain C element systems + textbook LU condensation) on the
    host cores, on a sample of the benchmark's elements."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    O.build()
    sz = O.Sizes(wl.mesh)
    cores = max(1, min(16, os.cpu_count() or 1))

    def one(e):
        E = O.element_system(wl, e, sz)
        O.condense(E, sz.n(e))

    # calibrate on one element, then size the sample to ~`seconds` of work
    t0 = time.perf_counter()
    one(0)
    t1 = time.perf_counter() - t0
    per_wave = max(t1, 1e-3)
    waves = max(1, int(seconds / per_wave))
    count = min(wl.mesh.n_elem, cores * waves)
    elems = list(range(count))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(one, elems))
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "elements/s", "cores": cores, "kind": "oracle",
            "sample": f"element residual+Jacobian and condensation of elements 0..{count - 1} "
                      f"({count} of {wl.mesh.n_elem}) of the same workload; trace assembly, Schwarz and GMRES "
                      f"excluded; {dt:.1f} s wall on {cores} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=1, choices=(1, 3, 4),
                    help="1: 8^3 p=3 supersonic TGV (the headline workload); 3: 2000 wall-stretched hexahedra "
                         "with p in {2,3,4}; 4: 12^3 p=4, chunks of 256, GMRES(50) with FP32 Schwarz, step "
                         "replayed from a HIP graph")
    ap.add_argument("--graph", action="store_true", help="also time the step replayed from a HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU's partition only (--gpus {args.gpus} requested); "
              "multi-GPU sharding is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2608_27863_amd import hdg, pipeline, synth

    big = args.config == 4
    use_graph = args.graph or big
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

    def timed(run_step):
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            run_step(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phase_ms = {ph: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(args.steps)]))
                    for i, ph in enumerate(phases)}
        return 1e3 * wall / args.steps, phase_ms

    def timed_graph(obj):
        graph = obj.capture()
        for _ in range(max(1, args.warmup)):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / args.steps

    def check(obj, what):
        if not np.all(obj.info.cpu().numpy() == 0) or not np.all(obj.asm_info.cpu().numpy() == 0):
            raise RuntimeError(f"zero pivot reported in the {what} warm-up")

    step = stepper(st)
    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    check(st, "FP64")
    ms_step, phase_ms = timed(step)
    print(f"[bench] {args.steps} timed steps: {ms_step:.2f} ms/step", file=sys.stderr, flush=True)
    graph_ms = timed_graph(st) if use_graph else None
    if graph_ms is not None:
        print(f"[bench] graph replay: {graph_ms:.2f} ms/step", file=sys.stderr, flush=True)
    S64 = None if big else st.S.clone()
    g64, d64 = st.g.clone(), st.dUhat.clone()

    # face matvec roofline (HBM): algorithmic bytes / kernel time, alternating buffers
    x0 = torch.as_tensor(wl.x, dtype=torch.float64, device="cuda")
    xs = [x0, x0.clone()]
    ys = [torch.empty_like(x0) for _ in range(2)]
    for _ in range(3):
        ctx.hdg_face_matvec(st.S, xs[0], ys[0])
    reps = 50
    mv_ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    mv_ev[0].record(stream)
    for r in range(reps):
        ctx.hdg_face_matvec(st.S, xs[r % 2], ys[r % 2])
        mv_ev[r + 1].record(stream)
    torch.cuda.synchronize()
    mv_ms = float(np.mean([mv_ev[r].elapsed_time(mv_ev[r + 1]) for r in range(reps)]))
    mv_bytes = matvec_bytes(ctx)
    mv_gbps = mv_bytes / (mv_ms * 1e-3) / 1e9

    # mixed-precision step on the same workload and context
    stm = pipeline.NewtonStep(wl, prec=hdg.HDG_MIXED, refine_steps=1, ctx=ctx, chunk=chunk,
                              share=st if big else None)
    step_mixed = stepper(stm)
    for w in range(args.warmup):
        step_mixed()
        torch.cuda.synchronize()
    check(stm, "mixed")
    ms_mixed, phase_mixed = timed(step_mixed)
    print(f"[bench] mixed: {ms_mixed:.2f} ms/step", file=sys.stderr, flush=True)
    graph_mixed = timed_graph(stm) if use_graph else None
    relnorm = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    mfl = [mixed_flops_per_element(a, b, 1) for a, b in zip(ns, fs)]
    f32tot, f64tot = sum(x[0] for x in mfl), sum(x[1] for x in mfl)
    t_cm = phase_mixed["condense"] * 1e-3
    t_peak = f32tot / (PEAK_FP32_TFLOPS * 1e12) + f64tot / (PEAK_FP64_TFLOPS * 1e12)
    mixed = {
        "value": ne / (ms_mixed * 1e-3), "unit": "elements/s", "ms_per_step": ms_mixed,
        "graph_ms_per_step": graph_mixed,
        "condense_elements_per_s": ne / t_cm, "phase_ms": phase_mixed,
        "refine_steps": 1, "schwarz": "element-block, FP32 inverses",
        "rel_diff_vs_fp64_step": {"S": None if S64 is None else relnorm(stm.S, S64), "g": relnorm(stm.g, g64),
                                  "dUhat_fixed_m": relnorm(stm.dUhat, d64)},
        "roofline": {"bound": "mfma", "time_at_peak_ms": 1e3 * t_peak, "frac": t_peak / t_cm,
                     "algorithmic": f"{f32tot:.4e} FP32 + {f64tot:.4e} FP64 flop over {ne} elements "
                                    f"(peaks {PEAK_FP32_TFLOPS} / {PEAK_FP64_TFLOPS} TFLOP/s)"},
    }

    # condensation roofline (FP64 matrix cores): dense algorithmic flops / hdg_condense time
    fl = sum(condense_flops_per_element(a, b) for a, b in zip(ns, fs))
    t_cond = phase_ms["condense"] * 1e-3
    achieved = fl / t_cond / 1e12
    tag = {1: "tgv8_p3", 3: "bl2000_p234", 4: "tgv12_p4"}[args.config]
    out = {
        "metric": "HDG condensed elements/s, FP64 vs mixed @1e-10 rel; face-matvec GB/s",
        "value": ne / (ms_step * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "elements": ne, "p": p,
                   "n_interior": n if len(degrees) == 1 else f"{min(ns)}-{max(ns)}",
                   "f_trace": f if len(degrees) == 1 else f"{min(fs)}-{max(fs)}",
                   "chunk": chunk or ne, "batches": [n for _, n in st.chunks], "gmres_iterations": st.m,
                   "schwarz": "element-block, " + ("FP32 inverses" if big else "FP64"), "precision": "FP64",
                   "step": f"residual+Jacobian, condensation, assembly, Schwarz set-up, GMRES({st.m}), recovery"},
        "graph_ms_per_step": graph_ms,
        "condense_elements_per_s": ne / t_cond,
        "phase_ms": phase_ms,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(f"condense_fp64_{tag}_hbm"),
                     "kernel": "hdg_condense (per pair of 128-column blocks: k_panel, k_half, k_crows, k_rowperm, k_inv128, k_blocku, "
                               "k_update; then k_extract)",
                     "algorithmic": f"{fl:.4e} flop over {ne} elements (LU 2n^3/3 + solve 2n^2(f+1) + "
                                    f"Schur 2fn(f+1) per element)"},
        "roofline_matvec": {"bound": "hbm", "achieved": mv_gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                            "frac": mv_gbps / PEAK_HBM_GBPS, "traffic": measured_traffic(f"matvec_{tag}_hbm"),
                            "kernel": "k_matvec", "ms": mv_ms, "algorithmic_bytes": mv_bytes},
        "mixed": mixed,
    }
    calibration_copy(torch)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
